// Host side of libqs: the C ABI declared in include/qs.h.
//
// Validation happens here before anything is enqueued; gates are brought to
// a canonical form (controls pulled out of the matrix, diagonal gates routed
// to the phase kernel) and launched on the state's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "qs_internal.h"
#include "qs_plan.h"
#include "qs_tile.h"
#include "qs_traj.h"
#include "qs_mlp.h"

#include <array>
#include <condition_variable>
#include <pthread.h>
#include <functional>
#include <mutex>
#include <shared_mutex>
#include <tuple>
#include "qs_philox.h"

#include <chrono>
#include <map>
#include <unordered_map>

using cd = std::complex<double>;

namespace {

// Text of the last failure on this thread, in a fixed buffer (recording an
// error allocates nothing).
thread_local char g_err[512];
std::atomic<size_t> g_mem_limit{0};

qs_status fail(qs_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

qs_status hip_fail(hipError_t e, const char *what)
{
    return fail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// Handlers of the function-try-block around every C ABI entry: no C++
// exception crosses the ABI (host allocation failures report QS_E_NOMEM).
#define QS_ABI_CATCH                                                              \
    catch (const std::bad_alloc &)                                                \
    {                                                                             \
        return fail(QS_E_NOMEM, "host allocation failed");                        \
    }                                                                             \
    catch (const std::exception &ex_)                                             \
    {                                                                             \
        return fail(QS_E_INVAL, "unexpected host exception: %s", ex_.what());     \
    }                                                                             \
    catch (...)                                                                   \
    {                                                                             \
        return fail(QS_E_INVAL, "unexpected host exception");                     \
    }

size_t amp_bytes(qs_dtype dt) { return dt == QS_C128 ? 16 : 8; }

struct ProfRec {
    int kid;
    hipEvent_t a, b;
    double bytes, flops;
    int feat;   // index into qs_state::feat_pending, or -1
    int n;
};

using Features = std::array<float, QS_COST_FEATURES>;

std::mutex g_model_mu;
std::vector<float> g_model;  // installed cost-model parameters (empty = none)

struct ProfAcc {
    int64_t launches = 0;
    double ms = 0, bytes = 0, flops = 0;
};

}  // namespace

struct qs_state {
    int n = 0;
    qs_dtype dt = QS_C128;
    int device = 0;
    void *amp = nullptr;
    size_t bytes = 0;
    bool owned = true;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double *red = nullptr;      // reduction scratch
    size_t red_doubles = 0;
    double *dout = nullptr;     // small device results (<= 64 KiB)
    void *dmat = nullptr;       // device staging for one gate matrix
    void *prog = nullptr;       // device matrices of a planned circuit segment
    size_t prog_bytes = 0;
    uint64_t prog_loaded = 0;   // id of the tile program resident in prog (0 = none)
    double *hpin = nullptr;     // pinned host results (64 KiB)
    bool prof = false;
    std::vector<Features> feat_pending;               // features of timed sweeps
    std::vector<std::pair<Features, float>> samples;  // (features, ln ns per amplitude)
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> pool;
    ProfAcc acc[QS_K_COUNT];
};

namespace {
struct CachedPlan;
struct PlanKey {
    int n, dt, plan, kmax, tile;
    uint64_t model;
    bool operator<(const PlanKey &o) const
    {
        return std::tie(n, dt, plan, kmax, tile, model) < std::tie(o.n, o.dt, o.plan, o.kmax, o.tile, o.model);
    }
};
std::atomic<uint64_t> g_model_version{1};
std::atomic<uint64_t> g_prog_serial{1};
}  // namespace

// Measured candidates of QS_PLAN_AUTOTUNE for one state shape.
struct Tuning {
    struct Cand {
        int tile, kmax;
        double seconds;  // < 0: not run yet
    };
    std::vector<Cand> cands;
    size_t next = 0;
    int best = -1;
};

struct qs_circuit {
    std::vector<qs::Op> ops;
    // plans already made for this circuit and autotuning records (cleared
    // when it changes)
    mutable std::mutex mu;
    mutable std::map<PlanKey, std::shared_ptr<const CachedPlan>> cache;
    mutable std::map<std::pair<int, int>, Tuning> tuning;
    mutable std::map<uint64_t, std::shared_ptr<const void>> other;  // plans of other modes (single-amplitude)
    void changed()
    {
        std::lock_guard<std::mutex> lk(mu);
        cache.clear();
        tuning.clear();
        other.clear();
    }
};

namespace {

// ------------------------------------------------------------ profiling --

hipEvent_t take_event(qs_state *s)
{
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

qs_status harvest(qs_state *s)
{
    for (auto &r : s->pending) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        auto &a = s->acc[r.kid];
        a.launches += 1;
        a.ms += ms;
        a.bytes += r.bytes;
        a.flops += r.flops;
        if (r.feat >= 0 && ms > 0)
            s->samples.push_back({s->feat_pending[r.feat], float(std::log(double(ms) * 1e6 / std::ldexp(1.0, r.n)))});
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->pending.clear();
    s->feat_pending.clear();
    return QS_OK;
}

struct Timed {
    qs_state *s;
    int kid;
    double bytes, flops;
    int feat = -1;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(qs_state *s_, int kid_, double bytes_, double flops_, const Features *f = nullptr)
        : s(s_), kid(kid_), bytes(bytes_), flops(flops_)
    {
        if (s->prof && f) {
            feat = int(s->feat_pending.size());
            s->feat_pending.push_back(*f);
        }
        if (s->prof) {
            if (s->pending.size() > 8192) harvest(s);
            a = take_event(s);
            b = take_event(s);
            if (a) hipEventRecord(a, s->stream);
        }
    }
    ~Timed()
    {
        if (s->prof && a && b) {
            hipEventRecord(b, s->stream);
            s->pending.push_back({kid, a, b, bytes, flops, feat, s->n});
        }
    }
};

// ----------------------------------------------------------- validation --

qs_status check_state(const qs_state *s)
{
    if (!s) return fail(QS_E_INVAL, "state is NULL");
    return QS_OK;
}

qs_status check_qubits(int n, const int *t, int nt, const int *c, int nc, int max_nt)
{
    if (nt < 1 || nt > max_nt) return fail(QS_E_INVAL, "number of targets %d not in [1, %d]", nt, max_nt);
    if (nc < 0) return fail(QS_E_INVAL, "negative number of controls");
    if (!t) return fail(QS_E_INVAL, "targets is NULL");
    if (nc > 0 && !c) return fail(QS_E_INVAL, "controls is NULL");
    if (nt + nc > n) return fail(QS_E_RANGE, "%d qubits named on a %d-qubit state", nt + nc, n);
    uint64_t seen = 0;
    for (int k = 0; k < nt + nc; ++k) {
        const int q = k < nt ? t[k] : c[k - nt];
        if (q < 0 || q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        if (seen >> q & 1) return fail(QS_E_RANGE, "qubit %d named twice", q);
        seen |= uint64_t(1) << q;
    }
    return QS_OK;
}

qs_status check_matrix(const double *m, int nt)
{
    if (!m) return fail(QS_E_INVAL, "matrix is NULL");
    const size_t len = size_t(2) << (2 * nt);
    for (size_t k = 0; k < len; ++k)
        if (!std::isfinite(m[k])) return fail(QS_E_INVAL, "matrix entry %zu is not finite", k / 2);
    return QS_OK;
}

qs_status check_kraus(const double *kr, int nk, int nt)
{
    if (!kr) return fail(QS_E_INVAL, "Kraus matrices are NULL");
    if (nk < 1 || nk > QS_MAX_KRAUS) return fail(QS_E_INVAL, "Kraus count %d not in [1, %d]", nk, QS_MAX_KRAUS);
    const int d = 1 << nt;
    const size_t blk = size_t(2) * d * d;
    for (size_t k = 0; k < blk * nk; ++k)
        if (!std::isfinite(kr[k])) return fail(QS_E_INVAL, "Kraus entry is not finite");
    // sum_b K_b^dagger K_b = I (Sec. 2.4)
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            cd s = 0;
            for (int b = 0; b < nk; ++b) {
                const double *K = kr + blk * b;
                for (int j = 0; j < d; ++j) {
                    cd kjr(K[2 * (j * d + r)], K[2 * (j * d + r) + 1]);
                    cd kjc(K[2 * (j * d + c)], K[2 * (j * d + c) + 1]);
                    s += std::conj(kjr) * kjc;
                }
            }
            const cd want = (r == c) ? 1.0 : 0.0;
            if (std::abs(s - want) > 1e-10)
                return fail(QS_E_INVAL, "Kraus set is not complete: (sum K^dagger K)[%d][%d] = %g%+gi", r, c,
                            s.real(), s.imag());
        }
    return QS_OK;
}

// ---------------------------------------------------------------- launch --

double flops_dense(int nt) { return 8.0 * double(1 << nt); }  // per amplitude

// Matrices of the 4-6 target kernels live in device memory.  A single gate
// waits for earlier work on the stream before it overwrites the staging
// buffer; a circuit uploads the matrices of a whole segment at once.
qs_status stage_matrix(qs_state *s, const qs::CanonGate &g)
{
    const int d = 1 << g.targets.size();
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->dt == QS_C128) {
        HIP_TRY(hipMemcpy(s->dmat, g.m.data(), size_t(16) * d * d, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(size_t(2) * d * d);
        for (size_t k = 0; k < f.size(); ++k) f[k] = float(g.m[k]);
        HIP_TRY(hipMemcpy(s->dmat, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return QS_OK;
}

// Launch one canonical gate.  Algorithmic bytes: every amplitude the kernel
// changes is read and written once.  dev_m: device copy of a 4-6 target
// matrix in the state's dtype (staged here when NULL).
qs_status launch_canon(qs_state *s, const qs::CanonGate &g, const void *dev_m = nullptr)
{
    const int n = s->n;
    const double ab = double(amp_bytes(s->dt));
    if (g.kind == qs::CanonGate::IDENTITY) return QS_OK;
    qs::IdxSpec ix{};
    int all[2 * qs::kMaxQ];
    int na = 0;
    for (int q : g.targets) all[na++] = q;
    for (int q : g.controls) all[na++] = q;
    std::sort(all, all + na);
    ix.npos = na;
    for (int k = 0; k < na; ++k) ix.pos[k] = all[k];
    ix.set = 0;
    for (int q : g.controls) ix.set |= uint64_t(1) << q;
    const int nt = int(g.targets.size());
    const double groups = std::ldexp(1.0, n - na);
    hipError_t e = hipSuccess;
    if (g.kind == qs::CanonGate::PHASE) {
        int active = 0;
        for (int x = 0; x < (1 << nt); ++x)
            if (!(g.m[2 * x] == 1.0 && g.m[2 * x + 1] == 0.0)) ++active;
        Timed t(s, QS_K_PHASE, 2.0 * ab * groups * active, 6.0 * groups * active);
        e = qs::launch_phase(s->dt, s->amp, n, ix, g.targets.data(), nt, g.m.data(), s->stream);
    } else if (nt == 1) {
        Timed t(s, QS_K_DENSE1, 2.0 * ab * groups * 2, flops_dense(1) * groups * 2);
        e = qs::launch_dense1(s->dt, s->amp, n, ix, g.targets[0], g.m.data(), s->stream);
    } else if (nt == 2) {
        Timed t(s, QS_K_DENSE2, 2.0 * ab * groups * 4, flops_dense(2) * groups * 4);
        e = qs::launch_dense2(s->dt, s->amp, n, ix, g.targets.data(), g.m.data(), s->stream);
    } else if (nt == 3) {
        Timed t(s, QS_K_DENSE3, 2.0 * ab * groups * 8, flops_dense(3) * groups * 8);
        e = qs::launch_dense3(s->dt, s->amp, n, ix, g.targets.data(), g.m.data(), s->stream);
    } else {
        const int d = 1 << nt;
        if (!dev_m) {
            if (qs_status st = stage_matrix(s, g)) return st;
            dev_m = s->dmat;
        }
        Timed t(s, QS_K_DENSEN, 2.0 * ab * groups * d, flops_dense(nt) * groups * d);
        e = qs::launch_denseN(s->dt, s->amp, n, ix, g.targets.data(), nt, dev_m, s->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "gate kernel launch");
    return QS_OK;
}

// Launch a planned segment: matrices of the 4-6 target gates are uploaded
// together first (after earlier users of the upload buffer have finished).
qs_status launch_plan(qs_state *s, const std::vector<qs::CanonGate> &plan)
{
    const size_t esz = s->dt == QS_C128 ? 16 : 8;
    std::vector<size_t> off(plan.size(), SIZE_MAX);
    size_t total = 0;
    for (size_t k = 0; k < plan.size(); ++k)
        if (plan[k].kind == qs::CanonGate::DENSE && plan[k].targets.size() >= 4) {
            off[k] = total;
            total += esz << (2 * plan[k].targets.size());
        }
    if (total) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (total > s->prog_bytes) {
            if (s->prog) HIP_TRY(hipFree(s->prog));
            s->prog = nullptr;
            s->prog_bytes = 0;
            HIP_TRY(hipMalloc(&s->prog, total));
            s->prog_bytes = total;
        }
        std::vector<unsigned char> host(total);
        for (size_t k = 0; k < plan.size(); ++k) {
            if (off[k] == SIZE_MAX) continue;
            const std::vector<double> &m = plan[k].m;
            if (s->dt == QS_C128) {
                std::memcpy(host.data() + off[k], m.data(), m.size() * sizeof(double));
            } else {
                float *f = reinterpret_cast<float *>(host.data() + off[k]);
                for (size_t j = 0; j < m.size(); ++j) f[j] = float(m[j]);
            }
        }
        HIP_TRY(hipMemcpy(s->prog, host.data(), total, hipMemcpyHostToDevice));
        s->prog_loaded = 0;
    }
    for (size_t k = 0; k < plan.size(); ++k) {
        const void *dm = off[k] == SIZE_MAX ? nullptr : static_cast<unsigned char *>(s->prog) + off[k];
        if (qs_status st = launch_canon(s, plan[k], dm)) return st;
    }
    return QS_OK;
}

qs_status apply_gate_host(qs_state *s, const int *t, int nt, const int *c, int nc, const double *m)
{
    qs::CanonGate g = qs::canonicalize(t, nt, c, nc, m);
    return launch_canon(s, g);
}

// ---------------------------------------------------------- tile sweeps --

uint16_t bf16_rne(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

float bf16_float(uint16_t h)
{
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Matrix-core operand fragments of a dense 2^k block (k = 4, 5), in the order
// the tile kernel's lanes read them: for the real form A (2D x 2D, D = 2^k,
// entries [[Re U, -Im U], [Im U, Re U]] per complex entry with re/im
// interleaved), fragment (mt, s) of lane l holds
// A[16 mt + l % 16][32 s + 8 (l / 16) + j], j < 8, as bfloat16 (hi),
// followed by the same layout of the remainders (lo).
void append_fragments(const std::vector<double> &m, int k, std::vector<uint16_t> &out)
{
    const int D = 1 << k, MT = 2 * D / 16, KS = 2 * D / 32;
    const size_t base = out.size();
    const size_t nfr = size_t(MT) * KS * 64 * 8;
    out.resize(base + 2 * nfr);
    for (int mt = 0; mt < MT; ++mt)
        for (int s2 = 0; s2 < KS; ++s2)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int row = 16 * mt + lane % 16, col = 32 * s2 + 8 * (lane / 16) + j;
                    const int r = row / 2, a = row % 2, c = col / 2, b = col % 2;
                    const double ur = m[2 * (size_t(r) * D + c)], ui = m[2 * (size_t(r) * D + c) + 1];
                    const double v = (a == 0) ? (b == 0 ? ur : -ui) : (b == 0 ? ui : ur);
                    const uint16_t h = bf16_rne(float(v));
                    const uint16_t l = bf16_rne(float(v - double(bf16_float(h))));
                    const size_t idx = ((size_t(mt) * KS + s2) * 64 + lane) * 8 + j;
                    out[base + idx] = h;
                    out[base + nfr + idx] = l;
                }
}

// Host work spread over threads: f(i) for i < count, in any order.  A fixed
// set of worker threads, started on first use and kept for the life of the
// process (intentionally never destroyed, so no thread outlives the objects
// it waits on), takes items of the most recently published job.  The caller
// works on its own job too and returns once every item is done, so nested
// or concurrent calls cannot deadlock: at worst the caller does the work
// itself.  A job lives on the heap, held by every thread that took it, so a
// worker that wakes after the job is finished only sees an exhausted counter.
// A child process forked after the pool started inherits none of its threads
// and possibly a locked mutex: there parallel_for runs serially.
std::atomic<bool> g_pool_forked{false};

class WorkerPool {
public:
    struct Job {
        std::function<void(size_t)> fn;
        size_t count = 0;
        std::atomic<size_t> next{0}, done{0};
        std::mutex mu;
        std::condition_variable cv;
    };

    static WorkerPool &get()
    {
        static WorkerPool *pool = new WorkerPool();
        return *pool;
    }

    size_t workers() const { return threads_.size(); }

    void run(size_t count, std::function<void(size_t)> fn)
    {
        auto job = std::make_shared<Job>();
        job->fn = std::move(fn);
        job->count = count;
        {
            std::lock_guard<std::mutex> lk(mu_);
            cur_ = job;
            ++serial_;
        }
        cv_.notify_all();
        work(*job);
        std::unique_lock<std::mutex> lk(job->mu);
        job->cv.wait(lk, [&] { return job->done.load() == job->count; });
    }

private:
    WorkerPool()
    {
        pthread_atfork(nullptr, nullptr, [] { g_pool_forked.store(true); });
        const size_t hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t nw = std::min<size_t>(hw, 16) - 1;
        for (size_t t = 0; t < nw; ++t) threads_.emplace_back([this] { loop(); });
        for (auto &th : threads_) th.detach();
    }

    static void work(Job &j)
    {
        for (size_t i = j.next.fetch_add(1); i < j.count; i = j.next.fetch_add(1)) {
            j.fn(i);
            if (j.done.fetch_add(1) + 1 == j.count) {
                std::lock_guard<std::mutex> lk(j.mu);
                j.cv.notify_all();
            }
        }
    }

    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return serial_ != seen; });
                seen = serial_;
                j = cur_;
            }
            if (j) work(*j);
        }
    }

    std::mutex mu_;
    std::condition_variable cv_;
    std::shared_ptr<Job> cur_;
    uint64_t serial_ = 0;
    std::vector<std::thread> threads_;
};

template <typename F>
void parallel_for(size_t count, F &&f)
{
    if (count < 8 || g_pool_forked.load() || WorkerPool::get().workers() == 0) {
        for (size_t i = 0; i < count; ++i) f(i);
        return;
    }
    WorkerPool::get().run(count, [&f](size_t i) { f(i); });
}

// Device ops of a tiled plan and where their operand data goes.  The data is
// kept in the per-step pieces it was built in and written once, by write(),
// straight into the buffer it is uploaded from (a batch's pinned staging
// area); materialize() gathers it into `data` for plans kept between runs.
struct TileProgram {
    std::vector<qs::TileOpDev> ops;
    std::vector<size_t> first;      // first op of each sweep step
    size_t units = 0;               // uint16 count of the operand data (a multiple of 8)
    std::vector<std::vector<uint16_t>> piece;        // per step
    std::vector<size_t> piece_at;                    // uint16 offset of each piece
    std::vector<const std::vector<uint32_t> *> table;  // per-lane offset tables
    std::vector<size_t> table_at;                    // uint16 offset of each table
    std::vector<uint16_t> data;     // materialize(): the whole operand data
    size_t bytes() const { return units * sizeof(uint16_t); }
    void write(uint16_t *dst) const;
    void materialize()
    {
        data.resize(units);
        write(data.data());
        piece.clear();
        piece.shrink_to_fit();
    }
};

void pad16(std::vector<uint16_t> &d)
{
    while (d.size() % 8) d.push_back(0);
}

// Matrix-core lane layout of a dense tile op.  The 32 lanes of one LDS read
// vary in the 4 column bits and in the op qubit at lpos[k - 3]; the 16 lanes
// of a write in the column bits only.  With image(p) the bank vector of tile
// bit p under the tile swizzle, reads are conflict-free when the five images
// have rank 5 and writes when the column images have rank 4 in their low four
// bits (banks seen mod 16).  `pos` holds the tile bits of the op qubits;
// returns the op qubit to place at lpos[k - 3] and the column bits.
int gf2_rank(uint32_t *v, int n)
{
    int r = 0;
    for (int bit = 0; bit < 5 && r < n; ++bit) {
        int piv = -1;
        for (int i = r; i < n; ++i)
            if (v[i] >> bit & 1) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        std::swap(v[r], v[piv]);
        for (int i = 0; i < n; ++i)
            if (i != r && (v[i] >> bit & 1)) v[i] ^= v[r];
        ++r;
    }
    return r;
}

void search_lane_layout(const std::vector<int> &pos, int m, int &lane_q, uint32_t &colmask)
{
    auto image = [](int p) { return qs::tile_swizzle(1u << p) & 31u; };
    uint32_t opm = 0;
    for (int p : pos) opm |= 1u << p;
    std::vector<int> group;
    for (int p = 0; p < m; ++p)
        if (!(opm >> p & 1)) group.push_back(p);
    const int ng = int(group.size());
    int best = -1;
    for (int a = 0; a < ng; ++a)
        for (int b = a + 1; b < ng; ++b)
            for (int c = b + 1; c < ng; ++c)
                for (int d = c + 1; d < ng; ++d) {
                    const int cols[4] = {group[a], group[b], group[c], group[d]};
                    uint32_t w[4];
                    for (int i = 0; i < 4; ++i) w[i] = image(cols[i]) & 15u;
                    const bool wok = gf2_rank(w, 4) == 4;
                    for (size_t q = 0; q < pos.size(); ++q) {
                        uint32_t r[5];
                        for (int i = 0; i < 4; ++i) r[i] = image(cols[i]);
                        r[4] = image(pos[q]);
                        const int score = (gf2_rank(r, 5) == 5) + 2 * wok;
                        if (score > best) {
                            best = score;
                            lane_q = int(q);
                            colmask = (1u << cols[0]) | (1u << cols[1]) | (1u << cols[2]) | (1u << cols[3]);
                            if (score == 3) return;
                        }
                    }
                }
}

// Per-lane LDS byte offsets of a dense tile op (layout in qs_tile.h).
std::vector<uint32_t> lane_offsets(const qs::TileOpDev &d)
{
    const int k = d.k, D = 1 << k, MT = 2 * D / 16, KS = 2 * D / 32;
    const int per = qs::tile_lane_offsets(k);
    std::vector<uint32_t> out(size_t(64) * per);
    auto offset = [&](int x) {
        uint32_t o = 0;
        for (int b = 0; b < k; ++b)
            if ((x >> (k - 1 - b)) & 1) o |= 1u << d.lpos[b];
        return o;
    };
    for (int lane = 0; lane < 64; ++lane) {
        uint32_t gl = 0;
        for (uint32_t mm = d.colmask, c = uint32_t(lane & 15); mm; mm &= mm - 1, c >>= 1)
            if (c & 1) gl |= mm & (~mm + 1);
        uint32_t *o = out.data() + size_t(lane) * per;
        for (int s2 = 0; s2 < KS; ++s2)
            for (int jj = 0; jj < 4; ++jj) *o++ = qs::tile_swizzle(gl | offset(16 * s2 + 4 * (lane >> 4) + jj)) << 3;
        for (int mt = 0; mt < MT; ++mt)
            for (int jj = 0; jj < 2; ++jj) *o++ = qs::tile_swizzle(gl | offset(8 * mt + 2 * (lane >> 4) + jj)) << 3;
    }
    return out;
}


// The layout depends only on the op's tile bits and the tile size: searched
// once per process and remembered (a few thousand keys at most).
void choose_lane_layout(const std::vector<int> &pos, int m, int &lane_q, uint32_t &colmask)
{
    static std::shared_mutex mu;
    static std::map<uint64_t, std::pair<int, uint32_t>> memo;  // (tile-bit set, m) -> (lane bit, columns)
    uint64_t key = uint64_t(m) << 32;
    for (int p : pos) key |= uint64_t(1) << p;
    std::pair<int, uint32_t> v;
    bool found = false;
    {
        std::shared_lock<std::shared_mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) {
            v = it->second;
            found = true;
        }
    }
    if (!found) {
        std::vector<int> sorted(pos);
        std::sort(sorted.begin(), sorted.end());
        int q = int(sorted.size()) - 3;
        uint32_t cm = 0;
        search_lane_layout(sorted, m, q, cm);
        v = std::make_pair(sorted[q], cm);
        std::unique_lock<std::shared_mutex> lk(mu);
        memo.emplace(key, v);
    }
    colmask = v.second;
    lane_q = int(std::find(pos.begin(), pos.end(), v.first) - pos.begin());
}

// The matrix of a k-qubit op with its qubits reordered: new qubit b is old
// qubit order[b] (index 0 = most significant bit).
std::vector<double> permute_matrix(const double *m, int k, const std::vector<int> &order)
{
    const int D = 1 << k;
    std::vector<int> idx(D);
    for (int x = 0; x < D; ++x) {
        int o = 0;
        for (int b = 0; b < k; ++b)
            if ((x >> (k - 1 - b)) & 1) o |= 1 << (k - 1 - order[b]);
        idx[x] = o;
    }
    std::vector<double> out(size_t(2) * D * D);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            out[2 * (size_t(r) * D + c)] = m[2 * (size_t(idx[r]) * D + idx[c])];
            out[2 * (size_t(r) * D + c) + 1] = m[2 * (size_t(idx[r]) * D + idx[c]) + 1];
        }
    return out;
}

// Device ops and operand data of one sweep; data_off counts from the start of
// this sweep's data (16-byte units).
void build_sweep_program(const qs::Sweep &sw, std::vector<qs::TileOpDev> &ops, std::vector<uint16_t> &data)
{
    const auto &Q = sw.Q;
    auto lpos = [&](int q) {
        for (size_t b = 0; b < Q.size(); ++b)
            if (Q[b] == q) return int(b);
        return -1;
    };
    for (const auto &op : sw.ops) {
        qs::TileOpDev d{};
        pad16(data);
        d.data_off = uint32_t(data.size() / 8);
        d.k = int(op.qubits.size());
        d.no = int(op.outer.size());
        for (int b = 0; b < d.k; ++b) d.lpos[b] = lpos(op.qubits[b]);
        for (int b = 0; b < d.no; ++b) d.opos[b] = op.outer[b];
        if (op.kind == qs::TileOp::DENSE) {
            d.kind = 0;
            d.skip = op.skip;
            // lane layout: the chosen op qubit moves to lpos[k - 3]
            std::vector<int> pos(d.lpos, d.lpos + d.k), order(d.k);
            int lane_q = d.k - 3;
            choose_lane_layout(pos, int(Q.size()), lane_q, d.colmask);
            for (int b = 0, o = 0; b < d.k; ++b) {
                if (b == d.k - 3) {
                    order[b] = lane_q;
                    continue;
                }
                if (o == lane_q) ++o;
                order[b] = o++;
            }
            for (int b = 0; b < d.k; ++b) d.lpos[b] = pos[order[b]];
            // column-tile index bits: the tile bits outside the op and its columns
            uint32_t opm = 0;
            for (int p : pos) opm |= 1u << p;
            uint32_t bm = ((1u << Q.size()) - 1u) & ~opm & ~d.colmask;
            for (int t = 0; t < 6; ++t, bm &= bm - 1) d.cimg[t] = bm ? qs::tile_swizzle(bm & (~bm + 1)) << 3 : 0u;
            // fragments of each distinct matrix once, then one copy per
            // outer pattern in pattern order
            const int D = 1 << d.k;
            const size_t per = size_t(2) * D * D;
            const size_t nd = op.m.size() / per;
            std::vector<uint16_t> distinct;
            for (size_t u = 0; u < nd; ++u)
                append_fragments(permute_matrix(op.m.data() + u * per, d.k, order), d.k, distinct);
            const size_t fs = distinct.size() / nd;  // uint16 per matrix, a multiple of 8
            d.frag_stride = uint32_t(fs / 8);
            const size_t P = size_t(1) << d.no;
            const size_t before = data.size();
            data.resize(before + P * fs);
            for (size_t p = 0; p < P; ++p) {
                const size_t u = op.pmap.empty() ? p : op.pmap[p];
                std::memcpy(data.data() + before + p * fs, distinct.data() + u * fs, fs * sizeof(uint16_t));
            }
            // the per-lane offset table is shared program-wide (build_tile_program)
        } else {
            // one table of 2^k complex64 entries per outer pattern, each
            // padded to whole 16-byte units
            d.kind = 1;
            const size_t D = size_t(1) << d.k, P = size_t(1) << d.no;
            const size_t per = std::max<size_t>(D, 2);
            d.frag_stride = uint32_t(per / 2);
            for (size_t p = 0; p < P; ++p)
                for (size_t x = 0; x < per; ++x) {
                    const size_t e = p * D + x;
                    const float re = x < D ? float(op.m[2 * e]) : 0.f, im = x < D ? float(op.m[2 * e + 1]) : 0.f;
                    uint32_t ur, ui;
                    std::memcpy(&ur, &re, 4);
                    std::memcpy(&ui, &im, 4);
                    data.push_back(uint16_t(ur));
                    data.push_back(uint16_t(ur >> 16));
                    data.push_back(uint16_t(ui));
                    data.push_back(uint16_t(ui >> 16));
                }
        }
        ops.push_back(d);
    }
    pad16(data);
}

// Programs of all sweep steps, built in parallel; the data stays in its
// pieces until written.
void build_tile_program(const std::vector<qs::PlanStep> &steps, TileProgram &tp)
{
    const size_t ns = steps.size();
    std::vector<std::vector<qs::TileOpDev>> pops(ns);
    tp.piece.assign(ns, {});
    parallel_for(ns, [&](size_t i) {
        if (steps[i].sweep) build_sweep_program(steps[i].sw, pops[i], tp.piece[i]);
    });
    tp.piece_at.assign(ns, 0);
    tp.first.clear();
    size_t nops = 0, ndata = 0;
    for (size_t i = 0; i < ns; ++i) {
        tp.first.push_back(nops);
        tp.piece_at[i] = ndata;
        nops += pops[i].size();
        ndata += tp.piece[i].size();
    }
    // per-lane LDS offset tables: one per distinct lane layout of the program
    // (block width, column bits and op bits packed into one key: 3 + 13 + 5 x 4
    // bits), placed after the sweeps' data; the tables themselves are computed
    // once per process
    static std::shared_mutex memo_mu;
    static std::unordered_map<uint64_t, std::vector<uint32_t>> memo;  // entries are never erased
    std::unordered_map<uint64_t, uint32_t> slot_of;                    // key -> table slot
    tp.table.clear();
    tp.table_at.clear();
    std::vector<uint32_t> op_slot(nops, UINT32_MAX);
    size_t dend = ndata;
    for (size_t i = 0, o = 0; i < ns; ++i)
        for (size_t j = 0; j < pops[i].size(); ++j, ++o) {
            const qs::TileOpDev &d = pops[i][j];
            if (d.kind != 0) continue;
            uint64_t key = uint64_t(d.k) | uint64_t(d.colmask) << 3;
            for (int b = 0; b < d.k; ++b) key |= uint64_t(d.lpos[b]) << (16 + 4 * b);
            auto it = slot_of.find(key);
            if (it == slot_of.end()) {
                const std::vector<uint32_t> *lo = nullptr;
                {
                    std::shared_lock<std::shared_mutex> lk(memo_mu);
                    auto m = memo.find(key);
                    if (m != memo.end()) lo = &m->second;
                }
                if (!lo) {
                    std::vector<uint32_t> v = lane_offsets(d);
                    std::unique_lock<std::shared_mutex> lk(memo_mu);
                    lo = &memo.emplace(key, std::move(v)).first->second;
                }
                it = slot_of.emplace(key, uint32_t(tp.table.size())).first;
                tp.table.push_back(lo);
                tp.table_at.push_back(dend);
                dend += lo->size() * 2;  // uint32 entries in uint16 units (multiples of 8)
            }
            op_slot[o] = it->second;
        }
    tp.ops.resize(nops);
    parallel_for(ns, [&](size_t i) {
        const uint32_t base = uint32_t(tp.piece_at[i] / 8);
        for (size_t j = 0; j < pops[i].size(); ++j) {
            const size_t o = tp.first[i] + j;
            qs::TileOpDev d = pops[i][j];
            d.data_off += base;
            if (op_slot[o] != UINT32_MAX) d.offs_off = uint32_t(tp.table_at[op_slot[o]] / 8);
            tp.ops[o] = d;
        }
    });
    tp.units = std::max<size_t>(dend, 8);
    if (tp.ops.empty()) tp.ops.resize(1);
}

void TileProgram::write(uint16_t *dst) const
{
    if (piece.empty() && !data.empty()) {
        std::memcpy(dst, data.data(), bytes());
        return;
    }
    // pieces are split into slices of at most 1 MiB so that a few large
    // steps do not serialise the copy
    struct Job { const uint16_t *src; size_t at, n; };
    std::vector<Job> jobs;
    const size_t slice = size_t(1) << 19;
    auto add = [&](const uint16_t *src, size_t at, size_t n) {
        for (size_t o = 0; o < n; o += slice) jobs.push_back({src + o, at + o, std::min(slice, n - o)});
    };
    size_t used = 0;
    for (size_t i = 0; i < piece.size(); ++i) {
        add(piece[i].data(), piece_at[i], piece[i].size());
        used = std::max(used, piece_at[i] + piece[i].size());
    }
    for (size_t t = 0; t < table.size(); ++t) {
        const size_t n = table[t]->size() * 2;
        add(reinterpret_cast<const uint16_t *>(table[t]->data()), table_at[t], n);
        used = std::max(used, table_at[t] + n);
    }
    if (used < units) std::memset(dst + used, 0, (units - used) * sizeof(uint16_t));
    parallel_for(jobs.size(), [&](size_t i) {
        std::memcpy(dst + jobs[i].at, jobs[i].src, jobs[i].n * sizeof(uint16_t));
    });
}

qs::TileParams tile_params(int n, const qs_run_opts &o)
{
    qs::TileParams tp;
    tp.m = o.tile_qubits ? o.tile_qubits : qs::default_tile_qubits(n);
    tp.m = std::min(tp.m, n);
    tp.L = 4;
    tp.kmax = (o.k_max >= 4 && o.k_max <= 5) ? o.k_max : 4;  // four-qubit blocks: cheapest per gate on the matrix cores
    return tp;
}

bool tiled_plan(const qs_state *s, const qs_run_opts &o)
{
    return o.plan != QS_PLAN_UNFUSED && s->dt == QS_C64 && s->n >= 10;
}

// Kernel arguments of one sweep: the global qubit of every local tile bit
// (the kernel spreads a thread's local offsets over them), the bits outside
// the tile that index the tiles, and tile order 0 (launch_steps may change it).
qs::TileArgs make_tile_args(const qs::Sweep &sw, int n)
{
    qs::TileArgs ta{};
    ta.m = int(sw.Q.size());
    ta.nops = int(sw.ops.size());
    const auto &Q = sw.Q;
    for (int b = 0; b < 16; ++b) ta.q[b] = uint8_t(b < ta.m ? Q[b] : 0);
    uint64_t qm = 0;
    for (int q : Q) qm |= uint64_t(1) << q;
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    ta.omask = all & ~qm;
    ta.nouter = __builtin_popcountll(ta.omask);
    return ta;
}

// Cost-model features of one tile sweep (all scaled to about [0, 1]).
Features sweep_features(const qs::Sweep &sw, int n, qs_dtype dt)
{
    Features f{};
    int d4 = 0, d5 = 0, ph = 0, outer = 0, skips = 0, work = 0;
    for (const auto &op : sw.ops) {
        if (op.kind == qs::TileOp::DENSE) {
            (op.qubits.size() >= 5 ? d5 : d4)++;
            work += 1 << op.qubits.size();
            if (op.skip) ++skips;
        } else {
            ++ph;
        }
        outer += int(op.outer.size());
    }
    const int m = int(sw.Q.size());
    f[0] = m / 13.f;
    f[1] = n / 36.f;
    f[2] = d4 / 16.f;
    f[3] = d5 / 16.f;
    f[4] = ph / 16.f;
    f[5] = outer / 32.f;
    f[6] = skips / 16.f;
    f[7] = sw.gates / 64.f;
    for (int i = 0; i < 6; ++i) f[8 + i] = (m - 1 - i >= 4) ? sw.Q[m - 1 - i] / float(n) : 0.f;
    f[14] = dt == QS_C64 ? 1.f : 0.f;
    f[15] = work / 256.f;
    return f;
}

// Tile parameters for a segment.  Without a cost model: the defaults.  With
// one (QS_PLAN_LEARNED): plan the segment for every candidate shape (tile
// qubits 11 to 13, block width 4 or 5), keep each shape's plan that the
// fixed estimate prefers, predict every sweep's time of those plans with the
// network on the device and keep the cheapest plan, unless the greedy plan
// (default shape) is predicted within 3% of it.
qs_status choose_tile_params(qs_state *s, const std::vector<qs::FlatOp> &flat, size_t k, size_t e,
                             const qs_run_opts &o, qs::TileParams &best, std::vector<qs::PlanStep> &best_steps)
{
    best = tile_params(s->n, o);
    std::vector<float> model;
    if (o.plan == QS_PLAN_LEARNED) {
        std::lock_guard<std::mutex> lk(g_model_mu);
        model = g_model;
    }
    if (model.empty()) {
        qs::plan_tiles(flat, k, e, s->n, best, best_steps);
        return QS_OK;
    }
    // every shape's whole plans from the tile-qubit search; within a shape
    // the fixed estimate picks one (it ranks plans of one shape well: same
    // tile size and block width, fewer sweeps against more blocks), and the
    // network chooses among the shapes, where that estimate cannot compare
    // (measured on the 34-qubit circuit: letting the network choose among
    // every variant of every shape picked a plan 16% slower than greedy)
    std::vector<qs::TileParams> shapes;
    for (int m = 11; m <= 13; ++m)
        for (int km = 4; km <= 5; ++km) {
            qs::TileParams tp;
            tp.m = std::min(m, s->n);
            tp.kmax = km;
            shapes.push_back(tp);
        }
    std::vector<std::vector<std::vector<qs::PlanStep>>> var(shapes.size());
    parallel_for(shapes.size(), [&](size_t i) { qs::plan_tiles_variants(flat, k, e, s->n, shapes[i], var[i]); });
    std::vector<qs::TileParams> cand;
    std::vector<std::vector<qs::PlanStep>> plans;
    size_t dflt = SIZE_MAX;  // the plan the fixed estimate picks at the default shape
    for (size_t i = 0; i < shapes.size(); ++i) {
        if (var[i].empty()) continue;
        size_t w = 0;
        for (size_t j = 1; j < var[i].size(); ++j)
            if (qs::plan_cost(var[i][j]) < qs::plan_cost(var[i][w])) w = j;
        if (shapes[i].m == best.m && shapes[i].kmax == best.kmax) dflt = plans.size();
        cand.push_back(shapes[i]);
        plans.push_back(std::move(var[i][w]));
    }
    std::vector<float> feats;
    std::vector<std::pair<int, int>> owner;  // (candidate, standalone?)
    for (size_t c = 0; c < cand.size(); ++c) {
        for (auto &st : plans[c]) {
            qs::Sweep sw = st.sweep ? st.sw : qs::Sweep{};
            if (!st.sweep) {  // a per-gate launch: scored as a sweep with one op
                sw.Q.assign(1, 0);
                sw.gates = 1;
            }
            const Features f = sweep_features(sw, s->n, s->dt);
            feats.insert(feats.end(), f.begin(), f.end());
            owner.push_back({int(c), st.sweep ? 0 : 1});
        }
    }
    const int64_t ns = int64_t(owner.size());
    float *dp = nullptr, *dx = nullptr, *dy = nullptr;
    std::vector<float> y(ns);
    hipError_t he = hipMalloc(&dp, model.size() * sizeof(float));
    if (he == hipSuccess) he = hipMalloc(&dx, feats.size() * sizeof(float));
    if (he == hipSuccess) he = hipMalloc(&dy, ns * sizeof(float));
    if (he == hipSuccess) he = hipMemcpy(dp, model.data(), model.size() * sizeof(float), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(dx, feats.data(), feats.size() * sizeof(float), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = qs::launch_mlp_forward(dp, QS_COST_FEATURES, qs::kMlpHidden, dx, ns, dy, s->stream);
    if (he == hipSuccess) he = hipMemcpyAsync(y.data(), dy, ns * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(s->stream);
    if (dp) (void)hipFree(dp);
    if (dx) (void)hipFree(dx);
    if (dy) (void)hipFree(dy);
    if (he != hipSuccess) return hip_fail(he, "cost-model inference");
    std::vector<double> cost(cand.size(), 0.0);
    for (int64_t i = 0; i < ns; ++i) cost[owner[i].first] += std::exp(double(y[i]));
    size_t bi = 0;
    for (size_t c = 1; c < cand.size(); ++c)
        if (cost[c] < cost[bi]) bi = c;
    // the greedy plan stands unless another is predicted clearly cheaper:
    // the network's errors on whole plans are a few percent
    constexpr double kMargin = 0.03;
    if (dflt != SIZE_MAX && cost[bi] > (1.0 - kMargin) * cost[dflt]) bi = dflt;
    best = cand[bi];
    best_steps = std::move(plans[bi]);
    return QS_OK;
}

// Upload a materialized tile program into the state's plan buffer unless it is already
// there (repeated runs of a cached plan skip the upload and its wait).
qs_status upload_program(qs_state *s, const TileProgram &tp, uint64_t id, size_t &doff)
{
    const size_t ob = tp.ops.size() * sizeof(qs::TileOpDev);
    const size_t db = tp.bytes();
    doff = ((ob + 255) / 256) * 256;
    if (id && s->prog_loaded == id) return QS_OK;
    const size_t total = doff + db;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (total > s->prog_bytes) {
        if (s->prog) HIP_TRY(hipFree(s->prog));
        s->prog = nullptr;
        s->prog_bytes = 0;
        HIP_TRY(hipMalloc(&s->prog, total));
        s->prog_bytes = total;
    }
    unsigned char *dev = static_cast<unsigned char *>(s->prog);
    HIP_TRY(hipMemcpy(dev, tp.ops.data(), ob, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dev + doff, tp.data.data(), db, hipMemcpyHostToDevice));
    s->prog_loaded = id;
    return QS_OK;
}

// Tile order of every sweep of one tiled segment (qs_run_opts.tile_order =
// 0).  The first QS_TILE_ORDERS runs of the segment each time all its sweeps
// under one candidate order; later runs take each sweep's fastest.  Shared by
// every state that runs the cached plan.
struct OrderTune {
    std::mutex mu;
    int next = 0;                                       // next candidate to time
    int done = 0;                                       // candidates timed
    std::vector<std::array<float, QS_TILE_ORDERS>> ms;  // per step
    std::vector<uint8_t> best;                          // per step, once every candidate is timed
};

// Events bracketing the sweeps of one timing run.
struct SweepEvents {
    std::vector<hipEvent_t> ev;
    ~SweepEvents()
    {
        for (hipEvent_t e : ev) hipEventDestroy(e);
    }
    hipError_t record(hipStream_t st)
    {
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        return hipEventRecord(e, st);
    }
};

qs_status launch_steps(qs_state *s, const std::vector<qs::PlanStep> &steps, const TileProgram &tp, uint64_t id,
                       OrderTune *tune, int fixed_order)
{
    size_t doff = 0;
    if (qs_status e = upload_program(s, tp, id, doff)) return e;
    unsigned char *dev = static_cast<unsigned char *>(s->prog);
    const qs::TileOpDev *dops = reinterpret_cast<const qs::TileOpDev *>(dev);
    const double sweep_bytes = 2.0 * 8.0 * std::ldexp(1.0, s->n);
    int cand = -1;  // candidate order timed by this run
    std::vector<uint8_t> best;
    if (fixed_order == 0 && tune) {
        std::lock_guard<std::mutex> lk(tune->mu);
        if (tune->next < QS_TILE_ORDERS)
            cand = tune->next++;
        else
            best = tune->best;  // empty while another run still times a candidate
    }
    SweepEvents sev;
    std::vector<size_t> timed;  // steps bracketed by sev, in order
    for (size_t i = 0; i < steps.size(); ++i) {
        const qs::PlanStep &st = steps[i];
        if (!st.sweep) {
            if (qs_status e = launch_canon(s, st.gate)) return e;
            continue;
        }
        qs::TileArgs ta = make_tile_args(st.sw, s->n);
        ta.order = fixed_order > 0 ? fixed_order - 1 : cand >= 0 ? cand : i < best.size() ? best[i] : 0;
        double flops = 0;
        for (const auto &op : st.sw.ops)
            flops += (op.kind == qs::TileOp::DENSE ? 8.0 * double(1 << op.qubits.size()) : 6.0) *
                     std::ldexp(1.0, s->n);
        const Features feat = sweep_features(st.sw, s->n, s->dt);
        Timed t(s, QS_K_TILE, sweep_bytes, flops, &feat);
        bool k5 = false;
        for (size_t o = 0; o < st.sw.ops.size(); ++o) {
            const qs::TileOpDev &d = tp.ops[tp.first[i] + o];
            k5 = k5 || (d.kind == 0 && d.k == 5);
        }
        if (cand >= 0) {
            if (hipError_t e = sev.record(s->stream)) return hip_fail(e, "timing a tile sweep");
            timed.push_back(i);
        }
        hipError_t e = qs::launch_tile(s->amp, s->n, ta, dops + tp.first[i], dev + doff, k5, s->stream);
        if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
        if (cand >= 0)
            if (hipError_t e2 = sev.record(s->stream)) return hip_fail(e2, "timing a tile sweep");
    }
    if (cand < 0 || timed.empty()) return QS_OK;
    // this run's candidate: read the sweep times and, after the last
    // candidate, keep the fastest order of every sweep
    if (hipError_t e = hipEventSynchronize(sev.ev.back())) return hip_fail(e, "timing a tile sweep");
    std::vector<float> ms(timed.size());
    for (size_t k = 0; k < timed.size(); ++k)
        if (hipError_t e = hipEventElapsedTime(&ms[k], sev.ev[2 * k], sev.ev[2 * k + 1]))
            return hip_fail(e, "timing a tile sweep");
    std::lock_guard<std::mutex> lk(tune->mu);
    if (tune->ms.size() < steps.size()) tune->ms.resize(steps.size());
    for (size_t k = 0; k < timed.size(); ++k) tune->ms[timed[k]][cand] = ms[k];
    if (++tune->done == QS_TILE_ORDERS) {
        tune->best.assign(steps.size(), 0);
        for (size_t i = 0; i < steps.size(); ++i)
            for (int c = 1; c < QS_TILE_ORDERS; ++c)
                if (tune->ms[i][c] < tune->ms[i][tune->best[i]]) tune->best[i] = uint8_t(c);
    }
    return QS_OK;
}

// ---------------------------------------------------------- plan cache --

struct SegPlan {
    bool tiled = false;
    std::vector<qs::PlanStep> steps;   // tiled segments
    TileProgram prog;
    uint64_t prog_id = 0;
    std::shared_ptr<OrderTune> tune;   // tiled segments: measured tile orders
    std::vector<qs::CanonGate> gates;  // per-gate and per-block plans
    bool has_noise = false;            // a noise site follows the gates
    qs::FlatOp noise;
};

struct CachedPlan {
    std::vector<SegPlan> segs;
};

// ------------------------------------------------------------ reductions --

qs_status rdm_host(qs_state *s, const int *tq, int nt, double *out /* 2*4^nt */)
{
    const double ab = double(amp_bytes(s->dt));
    {
        Timed t(s, QS_K_REDUCE, ab * std::ldexp(1.0, s->n), 8.0 * std::ldexp(1.0, s->n) * (1 << nt));
        hipError_t e = qs::launch_rdm(s->dt, s->amp, s->n, tq, nt, s->red, s->dout, s->stream);
        if (e != hipSuccess) return hip_fail(e, "rdm launch");
    }
    const size_t len = size_t(2) << (2 * nt);
    HIP_TRY(hipMemcpyAsync(s->hpin, s->dout, len * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::memcpy(out, s->hpin, len * sizeof(double));
    return QS_OK;
}

// Noise channel on the present (post-gate) state: Sec. 2.4 steps 1-3 with the
// branch weights p_b = Tr(K_b rho_T K_b^dagger) taken from the FP64 reduced
// density matrix of the targets (one read sweep), or directly as c_b when
// every K_b^dagger K_b = c_b I (then p_b does not depend on the state).
qs_status apply_channel(qs_state *s, const int *tq, int nt, const double *kr, int nk, double u,
                        int *chosen, double *pchosen)
{
    const int d = 1 << nt;
    const size_t blk = size_t(2) * d * d;
    std::vector<double> p(nk);
    std::vector<std::vector<cd>> KK(nk, std::vector<cd>(size_t(d) * d));
    bool scalar = true;
    std::vector<double> cb(nk);
    for (int b = 0; b < nk; ++b) {
        const double *K = kr + blk * b;
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                cd acc = 0;
                for (int j = 0; j < d; ++j)
                    acc += std::conj(cd(K[2 * (j * d + r)], K[2 * (j * d + r) + 1])) *
                           cd(K[2 * (j * d + c)], K[2 * (j * d + c) + 1]);
                KK[b][size_t(r) * d + c] = acc;
            }
        cb[b] = KK[b][0].real();
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                const cd want = (r == c) ? cd(cb[b]) : cd(0);
                if (std::abs(KK[b][size_t(r) * d + c] - want) > 1e-14) scalar = false;
            }
    }
    if (scalar) {
        for (int b = 0; b < nk; ++b) p[b] = cb[b];
    } else {
        if (nt > 2) return fail(QS_E_UNSUPPORTED, "state-dependent Kraus sets on more than 2 qubits");
        std::vector<double> rho(size_t(2) * d * d);
        qs_status st = rdm_host(s, tq, nt, rho.data());
        if (st) return st;
        for (int b = 0; b < nk; ++b) {
            // Tr(K^dagger K rho) = sum_{y,x} (K^dagger K)_{y x} rho_{x y}
            cd tr = 0;
            for (int y = 0; y < d; ++y)
                for (int x = 0; x < d; ++x)
                    tr += KK[b][size_t(y) * d + x] * cd(rho[2 * (x * d + y)], rho[2 * (x * d + y) + 1]);
            p[b] = tr.real();
        }
    }
    int pick = -1;
    double run = 0.0;
    for (int b = 0; b < nk; ++b) {
        run += p[b];
        if (u < run) {
            pick = b;
            break;
        }
    }
    if (pick < 0)
        for (int b = nk - 1; b >= 0; --b)
            if (p[b] > 0) {
                pick = b;
                break;
            }
    if (pick < 0 || !(p[pick] > 0)) return fail(QS_E_ZERO_NORM, "every Kraus branch has probability 0");
    const double sc = 1.0 / std::sqrt(p[pick]);
    std::vector<double> m(blk);
    const double *K = kr + blk * pick;
    bool ident = true;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const size_t k = size_t(r) * d + c;
            m[2 * k] = K[2 * k] * sc;
            m[2 * k + 1] = K[2 * k + 1] * sc;
            const double want = (r == c) ? 1.0 : 0.0;
            if (std::abs(m[2 * k] - want) > 1e-14 || std::abs(m[2 * k + 1]) > 1e-14) ident = false;
        }
    if (chosen) *chosen = pick;
    if (pchosen) *pchosen = p[pick];
    // K_b / sqrt(p_b) equal to the identity up to 1e-14 (a scaled identity
    // branch): the renormalised state is the present one.
    if (ident) return QS_OK;
    return apply_gate_host(s, tq, nt, nullptr, 0, m.data());
}

qs_status alloc_state_buffers(qs_state *s)
{
    s->red_doubles = qs::reduce_scratch_doubles(s->n, 1024);
    HIP_TRY(hipMalloc(&s->red, s->red_doubles * sizeof(double)));
    HIP_TRY(hipMalloc(&s->dout, 65536));
    HIP_TRY(hipMalloc(&s->dmat, size_t(16) << (2 * QS_MAX_TARGETS)));
    HIP_TRY(hipHostMalloc((void **)&s->hpin, 65536, hipHostMallocDefault));
    return QS_OK;
}

void free_state(qs_state *s)
{
    if (!s) return;
    if (s->stream) hipStreamSynchronize(s->stream);
    for (auto &r : s->pending) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : s->pool) hipEventDestroy(e);
    if (s->owned && s->amp) hipFree(s->amp);
    if (s->red) hipFree(s->red);
    if (s->dout) hipFree(s->dout);
    if (s->dmat) hipFree(s->dmat);
    if (s->prog) hipFree(s->prog);
    if (s->hpin) hipHostFree(s->hpin);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    delete s;
}

qs_status init_amplitudes(qs_state *s)
{
    const uint64_t na = uint64_t(1) << s->n;
    Timed t(s, QS_K_INIT, double(amp_bytes(s->dt)) * double(na), 0.0);
    hipError_t e = qs::launch_init(s->dt, s->amp, na, s->stream);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    return QS_OK;
}

qs_status create_common(int n, qs_dtype dt, qs_state **out)
{
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS) return fail(QS_E_INVAL, "n = %d not in [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", int(dt));
    return QS_OK;
}

}  // namespace


// =============================================================== batches ==
//
// Noisy trajectories (Sec. 2.4), many states at once.  Per trajectory the
// circuit is cut into steps that alternate GATES, RUN, GATES, ..., GATES:
//  - GATES: gates, with every noise site whose branch weights do not depend
//    on the state (all K_b^dagger K_b = c_b I, e.g. depolarizing) already
//    sampled on the host from its Philox draw and replaced by K_b / sqrt(c_b);
//    a GATES step that follows a RUN begins with the RUN's K1 factors, the
//    operators of the path on which no site of the run jumps;
//  - RUN: consecutive one-qubit sites on distinct qubits whose first Kraus
//    operator is K1 = diag(1, k) (amplitude and phase damping), sampled
//    together from the prefix sums of one FP64 reduction pass (qs_traj.hip).
// Branch weights are ratios of those sums, so the K1 factors are applied
// without renormalising; a jump (K2) renormalises the state.
//
// Complex64 states of at least 10 qubits run in device-sampled passes: every
// remaining step of every trajectory is planned on the host, uploaded once,
// and executed as one captured HIP graph of batched tile sweeps, batched run
// sums and a sampling kernel that draws each site's Philox uniform on the
// device.  A trajectory whose run takes K2 at some site is frozen there (its
// later launches exit at once); after the pass the host rewrites its steps
// from the jump on (K1 of the earlier sites, K2, renormalisation, the rest
// of the run) and runs the frozen trajectories in the next pass.  Other
// states (complex128, fewer qubits, gates too wide for a tile) take the
// host-sampled path: one batched step at a time, run sums read back and
// sampled on the host.

namespace {

struct RunSite {
    int q;
    uint64_t site;
    std::vector<double> kraus;  // nk 2x2 matrices (K1 first)
    int nk;
    double a;                   // |K1_11|^2
};

struct TStep {
    bool run = false;
    std::vector<qs::FlatOp> gates;  // GATES: the first k1_lead are the K1 factors of the RUN before it
    int k1_lead = 0;
    std::vector<RunSite> sites;     // RUN
};

struct TPrep {
    int n = 0;
    std::vector<TStep> steps;
    size_t cur = 0;  // next step to execute
};

bool scalar_channel(const std::vector<double> &kr, int nk, int nt, std::vector<double> &c)
{
    const int d = 1 << nt;
    const size_t blk = size_t(2) * d * d;
    c.assign(nk, 0.0);
    for (int b = 0; b < nk; ++b) {
        const double *K = kr.data() + blk * b;
        std::vector<cd> kk(size_t(d) * d);
        for (int r = 0; r < d; ++r)
            for (int cc = 0; cc < d; ++cc) {
                cd acc = 0;
                for (int j = 0; j < d; ++j)
                    acc += std::conj(cd(K[2 * (j * d + r)], K[2 * (j * d + r) + 1])) * cd(K[2 * (j * d + cc)], K[2 * (j * d + cc) + 1]);
                kk[size_t(r) * d + cc] = acc;
            }
        c[b] = kk[0].real();
        for (int r = 0; r < d; ++r)
            for (int cc = 0; cc < d; ++cc)
                if (std::abs(kk[size_t(r) * d + cc] - ((r == cc) ? cd(c[b]) : cd(0))) > 1e-14) return false;
    }
    return true;
}

// scalar_channel for trajectory preparation: a circuit repeats a few
// channels at many sites, and the answer depends only on the Kraus
// matrices, so the last few answers are kept per thread (compared by
// content; the K_b^dagger K_b products of a two-qubit depolarizing channel
// are otherwise most of a trajectory's preparation).
bool scalar_channel_cached(const std::vector<double> &kr, int nk, int nt, std::vector<double> &c)
{
    struct Entry {
        int nk = -1, nt = -1;
        bool ok = false;
        std::vector<double> kr, c;
    };
    constexpr int kEntries = 4;
    thread_local Entry cache[kEntries];
    thread_local int next = 0;
    for (const Entry &e : cache)
        if (e.nk == nk && e.nt == nt && e.kr.size() == kr.size() &&
            std::memcmp(e.kr.data(), kr.data(), kr.size() * sizeof(double)) == 0) {
            c = e.c;
            return e.ok;
        }
    Entry &e = cache[next];
    next = (next + 1) % kEntries;
    e.ok = scalar_channel(kr, nk, nt, e.c);
    e.nk = nk;
    e.nt = nt;
    e.kr = kr;
    c = e.c;
    return e.ok;
}

// two one-qubit Kraus operators, K1 = diag(1, k), K2 acting only on |1>
bool damping_channel(const std::vector<double> &kr, int nk, int nt, double &a)
{
    if (nt != 1 || nk != 2) return false;
    const double *K1 = kr.data(), *K2 = kr.data() + 8;
    if (K1[0] != 1.0 || K1[1] != 0.0 || K1[2] != 0.0 || K1[3] != 0.0 || K1[4] != 0.0 || K1[5] != 0.0) return false;
    if (K2[0] != 0.0 || K2[1] != 0.0 || K2[4] != 0.0 || K2[5] != 0.0) return false;
    a = K1[6] * K1[6] + K1[7] * K1[7];
    return true;
}

int pick_branch(const std::vector<double> &p, double u)
{
    double run = 0.0;
    for (size_t b = 0; b < p.size(); ++b) {
        run += p[b];
        if (u < run) return int(b);
    }
    for (int b = int(p.size()) - 1; b >= 0; --b)
        if (p[b] > 0) return b;
    return -1;
}

qs::FlatOp one_qubit(int q, const double *m2)
{
    qs::FlatOp f;
    f.targets = {q};
    f.m.assign(m2, m2 + 8);
    return f;
}

qs_status prepare_trajectory(const qs_circuit *c, int n, uint64_t seed, uint64_t traj, TPrep &tp)
{
    std::vector<qs::FlatOp> flat;
    std::string err;
    int rc = qs::expand(c->ops, flat, err);
    if (rc) return fail(rc == 2 ? QS_E_UNSUPPORTED : QS_E_INVAL, "%s", err.c_str());
    tp.n = n;
    tp.cur = 0;
    TStep cur;
    bool since_run_only_identity = false;  // no non-identity gate since the open RUN
    uint64_t site = 0;
    for (auto &f : flat) {
        for (int q : f.targets)
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        for (int q : f.controls)
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        if (f.kind == qs::FlatOp::GATE) {
            if (!qs::is_identity(f.m, int(f.targets.size()))) since_run_only_identity = false;
            cur.gates.push_back(std::move(f));
            continue;
        }
        const int nt = int(f.targets.size());
        const double u = qs::noise_uniform(seed, traj, site);
        std::vector<double> cb;
        double a = 0;
        if (scalar_channel_cached(f.m, f.nk, nt, cb)) {
            const int b = pick_branch(cb, u);
            if (b < 0) return fail(QS_E_ZERO_NORM, "every Kraus branch has probability 0");
            const int d = 1 << nt;
            const size_t blk = size_t(2) * d * d;
            const double sc = 1.0 / std::sqrt(cb[b]);
            qs::FlatOp g;
            g.targets = f.targets;
            g.m.assign(f.m.begin() + blk * b, f.m.begin() + blk * (b + 1));
            bool ident = true;
            for (int r = 0; r < d; ++r)
                for (int cc = 0; cc < d; ++cc) {
                    const size_t k = size_t(r) * d + cc;
                    g.m[2 * k] *= sc;
                    g.m[2 * k + 1] *= sc;
                    if (std::abs(g.m[2 * k] - (r == cc ? 1.0 : 0.0)) > 1e-14 || std::abs(g.m[2 * k + 1]) > 1e-14) ident = false;
                }
            if (!ident) {
                cur.gates.push_back(std::move(g));
                since_run_only_identity = false;
            }
        } else if (damping_channel(f.m, f.nk, nt, a)) {
            qs::FlatOp k1 = one_qubit(f.targets[0], f.m.data());
            RunSite rs{f.targets[0], site, f.m, f.nk, a};
            TStep *last = tp.steps.empty() ? nullptr : &tp.steps.back();
            bool join = last && last->run && since_run_only_identity && int(last->sites.size()) < qs::kRunMax;
            if (join)
                for (auto &o : last->sites)
                    if (o.q == rs.q) join = false;
            if (join) {
                cur.gates.resize(size_t(cur.k1_lead));  // identity carriers only besides the run's K1 factors
                last->sites.push_back(std::move(rs));
            } else {
                tp.steps.push_back(std::move(cur));
                cur = TStep();
                TStep r;
                r.run = true;
                r.sites.push_back(std::move(rs));
                tp.steps.push_back(std::move(r));
            }
            cur.gates.push_back(std::move(k1));
            ++cur.k1_lead;
            since_run_only_identity = true;
        } else {
            return fail(QS_E_UNSUPPORTED, "batched trajectories support noise channels with state-independent "
                                          "weights and damping-type one-qubit channels");
        }
        ++site;
    }
    tp.steps.push_back(std::move(cur));
    return QS_OK;
}

// Site j of the RUN step r took K2 with branch weight nrm2 (the squared norm
// after K1 on sites 0..j-1 and K2 on site j): step r becomes the GATES step
// {K1 of sites < j, K2 of site j, 1/sqrt(nrm2)}, followed by a RUN of the
// sites after j (if any); the GATES step after the run loses the K1 factors
// of sites 0..j.  The trajectory continues at step r.
void jump_continuation(TPrep &tp, size_t r, size_t j, double nrm2)
{
    TStep g;
    TStep rest;
    rest.run = true;
    {
        const TStep &R = tp.steps[r];
        for (size_t i = 0; i < j; ++i) g.gates.push_back(one_qubit(R.sites[i].q, R.sites[i].kraus.data()));
        g.gates.push_back(one_qubit(R.sites[j].q, R.sites[j].kraus.data() + 8));
        const double sc = 1.0 / std::sqrt(nrm2);
        const double m2[8] = {sc, 0, 0, 0, 0, 0, sc, 0};
        g.gates.push_back(one_qubit(R.sites[j].q, m2));
        rest.sites.assign(R.sites.begin() + long(j) + 1, R.sites.end());
    }
    TStep &N = tp.steps[r + 1];  // the GATES step after a RUN always exists
    N.gates.erase(N.gates.begin(), N.gates.begin() + long(j) + 1);
    N.k1_lead -= int(j) + 1;
    tp.steps[r] = std::move(g);
    if (!rest.sites.empty()) tp.steps.insert(tp.steps.begin() + long(r) + 1, std::move(rest));
    tp.cur = r;
}

// A lightweight view of one trajectory's amplitudes that borrows the
// scratch buffers of a master state (all work is on one stream).
struct View {
    qs_state s;
    View(const qs_state *master, void *amp, int n)
    {
        s.n = n;
        s.dt = master->dt;
        s.device = master->device;
        s.amp = amp;
        s.owned = false;
        s.stream = master->stream;
        s.red = master->red;
        s.dout = master->dout;
        s.dmat = master->dmat;
        s.hpin = master->hpin;
    }
    ~View()
    {
        s.red = nullptr;
        s.dout = nullptr;
        s.dmat = nullptr;
        s.hpin = nullptr;
        s.prog = nullptr;
    }
};

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
        }
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) cap = bytes;
        return e;
    }
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Pinned host memory for uploads, grown on demand.
struct PinnedBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipHostFree(p);
            if (e != hipSuccess) return e;
        }
        p = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
        if (e == hipSuccess) cap = bytes;
        return e;
    }
    ~PinnedBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

// Tile planning of a trajectory's gate lists (planned once, never reused).
struct TrajParams {
    int m_cap = 13;     // qubits per tile (at most the state's width)
    int kmax = 4;       // widest dense block
    int max_outer = 1;  // outer selector bits per op
    int chunk = 128;    // trajectories per device-sampled job at most (0 = all waiting at once)
};

// Device buffers, host staging and the graph of one device-sampled pass
// job; a batch keeps two, so that the host builds the next job while the
// device runs the current one.
struct PassSlot {
    DevBuf prog, work;
    PinnedBuf stage, back;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
    bool busy = false;            // launched, results not yet read
    std::vector<int> set;         // the job's trajectories
    std::vector<char> out;        // per trajectory: plan needs per-gate launches (host-sampled path)
    size_t zb = 0, err_at = 0;    // read-back layout: freeze records, error flag, final sums
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~PassSlot()
    {
        drop_graph();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (done) (void)hipEventDestroy(done);
    }
};

// Pass slots outlive a batch: their device buffers, pinned staging buffers
// and events are allocated by the first batches on a device and reused by
// later ones (pinning a staging buffer of a hundred megabytes costs tens of
// milliseconds, a large share of a batch).  One idle pair is kept per device
// until the process ends; a batch that finds none (another thread holds it)
// makes its own.
std::mutex g_slot_mu;
std::map<int, std::unique_ptr<PassSlot[]>> *g_slot_pool = new std::map<int, std::unique_ptr<PassSlot[]>>;

std::unique_ptr<PassSlot[]> take_slots(int dev)
{
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        auto it = g_slot_pool->find(dev);
        if (it != g_slot_pool->end() && it->second) return std::move(it->second);
    }
    return std::unique_ptr<PassSlot[]>(new PassSlot[2]);
}

// Only after every job of the batch has finished (its stream has drained).
void give_slots(int dev, std::unique_ptr<PassSlot[]> p)
{
    for (int i = 0; i < 2; ++i) {
        p[i].drop_graph();
        p[i].busy = false;
        p[i].set.clear();
        p[i].out.clear();
    }
    std::lock_guard<std::mutex> lk(g_slot_mu);
    auto &q = (*g_slot_pool)[dev];
    if (!q) q = std::move(p);
}

struct Batch {
    qs_state *master = nullptr;  // scratch and stream owner (a 1-qubit state)
    qs_dtype dt;
    TrajParams par;
    bool graph = true;           // device-sampled passes run as captured HIP graphs
    uint64_t seed = 0;
    std::vector<TPrep> prep;
    std::vector<void *> amp;
    std::vector<size_t> zoff;    // offset of each trajectory's <Z_q> in the output
    double *z_out = nullptr;
    DevBuf states, prog, red, work;
    PinnedBuf stage, back;       // uploads (written only after the stream has drained), read-backs
    std::vector<View *> views;
    const qs_circuit *const *circs = nullptr;  // the call's circuits and widths
    const int *widths = nullptr;
    std::vector<char> ready;   // trajectory prepared (prepare_some)
    int dev = 0;
    std::unique_ptr<PassSlot[]> slot;  // two, from take_slots
    bool grew = false;                 // a job had to enlarge a slot's buffers
    qs_traj_stats st{};
    ~Batch()
    {
        if (master) (void)hipStreamSynchronize(master->stream);  // no buffer is freed under a running kernel
        for (auto *v : views) delete v;
        if (master) free_state(master);
        if (slot) give_slots(dev, std::move(slot));
    }
};

bool device_sampled(const Batch &B, int t) { return B.dt == QS_C64 && B.prep[t].n >= 10; }

// Prepare the trajectories of `ts` not prepared yet, in parallel (each job's
// just before it is built, so that preparing the rest of the batch overlaps
// the device's work on the first jobs); the first failure is reported on
// the calling thread.
qs_status prepare_some(Batch &B, const std::vector<int> &ts)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<int> todo;
    for (int t : ts)
        if (!B.ready[size_t(t)]) todo.push_back(t);
    std::vector<qs_status> pst(todo.size(), QS_OK);
    parallel_for(todo.size(), [&](size_t i) {
        const int t = todo[i];
        pst[i] = prepare_trajectory(B.circs[t], B.widths[t], B.seed, uint64_t(t), B.prep[t]);
    });
    for (size_t i = 0; i < todo.size(); ++i) {
        const int t = todo[i];
        if (pst[i] != QS_OK) {  // again on this thread, which reports the error
            B.prep[t] = TPrep();
            return prepare_trajectory(B.circs[t], B.widths[t], B.seed, uint64_t(t), B.prep[t]);
        }
        B.ready[size_t(t)] = 1;
    }
    B.st.host_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return QS_OK;
}

// Plan one gate list of a trajectory: tile sweeps for complex64 states of at
// least 10 qubits (gates wider than a tile block stay per-gate steps), the
// per-gate kernels otherwise.
void plan_gate_list(const Batch &B, int n, const std::vector<qs::FlatOp> &fl, std::vector<qs::PlanStep> &out)
{
    if (fl.empty()) return;
    if (B.dt == QS_C64 && n >= 10) {
        qs::TileParams tp;
        tp.m = std::min(B.par.m_cap, n);
        tp.L = 4;
        tp.kmax = B.par.kmax;
        tp.max_outer = B.par.max_outer;
        tp.search = false;  // planned once per trajectory step: keep it cheap
        qs::plan_tiles(fl, 0, fl.size(), n, tp, out);
        return;
    }
    for (auto &f : fl) {
        qs::PlanStep st;
        st.sweep = false;
        st.gate = qs::canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(), int(f.controls.size()),
                                   f.m.data());
        if (st.gate.kind != qs::CanonGate::IDENTITY) out.push_back(std::move(st));
    }
}

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// ------------------------------------------------------ host-sampled path --

// Apply one gate list to each listed trajectory: tiled complex64 plans run as
// batched sweep rounds, everything else through the per-gate kernels.
qs_status batch_gates(Batch &B, const std::vector<int> &who, const std::vector<const std::vector<qs::FlatOp> *> &lists)
{
    std::vector<std::vector<qs::PlanStep>> plans(who.size());
    parallel_for(who.size(), [&](size_t i) { plan_gate_list(B, B.prep[who[i]].n, *lists[i], plans[i]); });
    size_t rounds = 0;
    for (auto &pl : plans) rounds = std::max(rounds, pl.size());
    // flatten in (round, trajectory) order and build one device program
    std::vector<qs::PlanStep> all;
    struct Ref { size_t round; size_t who; };
    std::vector<Ref> refs;
    for (size_t r = 0; r < rounds; ++r)
        for (size_t i = 0; i < who.size(); ++i)
            if (r < plans[i].size()) {
                all.push_back(std::move(plans[i][r]));
                refs.push_back({r, i});
            }
    if (all.empty()) return QS_OK;
    TileProgram tp;
    build_tile_program(all, tp);
    std::vector<qs::TileArgsDev> args;
    std::vector<std::vector<qs::TileTask>> tasks(rounds * 4);  // per round, per m - 10
    for (size_t k = 0; k < all.size(); ++k) {
        if (!all[k].sweep) continue;
        const int t = who[refs[k].who];
        qs::TileArgsDev ad{};
        ad.amp = static_cast<float2 *>(B.amp[t]);
        ad.op_off = uint32_t(tp.first[k]);
        ad.ta = make_tile_args(all[k].sw, B.prep[t].n);
        args.push_back(ad);
        const uint32_t ntiles = uint32_t(1) << (B.prep[t].n - ad.ta.m);
        auto &tl = tasks[refs[k].round * 4 + (ad.ta.m - 10)];
        for (uint32_t tile = 0; tile < ntiles; ++tile) tl.push_back({uint32_t(args.size() - 1), tile});
    }
    size_t ntask = 0;
    for (auto &tl : tasks) ntask += tl.size();
    const size_t ob = tp.ops.size() * sizeof(qs::TileOpDev);
    const size_t db = tp.bytes();
    const size_t ab = args.size() * sizeof(qs::TileArgsDev);
    const size_t total = align256(ob) + align256(db) + align256(ab) + align256(ntask * sizeof(qs::TileTask)) + 256;
    qs_state *s = B.master;
    // the previous round's upload and kernels are done before the staging
    // buffer and the program buffer are rewritten
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(B.prog.ensure(total));
    HIP_TRY(B.stage.ensure(total));
    unsigned char *dev = static_cast<unsigned char *>(B.prog.p);
    unsigned char *host = static_cast<unsigned char *>(B.stage.p);
    std::vector<size_t> task_off(tasks.size());
    size_t toff = 0;
    for (size_t k = 0; k < tasks.size(); ++k) {
        task_off[k] = toff;
        toff += tasks[k].size();
    }
    const size_t o_data = align256(ob), o_args = o_data + align256(db), o_tasks = o_args + align256(ab);
    std::memcpy(host, tp.ops.data(), ob);
    tp.write(reinterpret_cast<uint16_t *>(host + o_data));
    if (ab) std::memcpy(host + o_args, args.data(), ab);
    for (size_t k = 0; k < tasks.size(); ++k)
        if (!tasks[k].empty())
            std::memcpy(host + o_tasks + task_off[k] * sizeof(qs::TileTask), tasks[k].data(),
                        tasks[k].size() * sizeof(qs::TileTask));
    HIP_TRY(hipMemcpyAsync(dev, host, o_tasks + ntask * sizeof(qs::TileTask), hipMemcpyHostToDevice, s->stream));
    const qs::TileOpDev *dops = reinterpret_cast<const qs::TileOpDev *>(dev);
    const qs::TileArgsDev *dargs = reinterpret_cast<const qs::TileArgsDev *>(dev + o_args);
    const qs::TileTask *dtasks = reinterpret_cast<const qs::TileTask *>(dev + o_tasks);
    bool k5 = false;  // any 5-qubit block selects the 256-thread kernel for every launch
    for (const auto &d : tp.ops) k5 = k5 || (d.kind == 0 && d.k == 5);
    size_t k = 0;
    for (size_t r = 0; r < rounds; ++r) {
        // standalone gates of this round (different states: any order)
        for (size_t kk = k; kk < all.size() && refs[kk].round == r; ++kk) {
            if (all[kk].sweep) continue;
            const int t = who[refs[kk].who];
            if (qs_status e = launch_canon(&B.views[t]->s, all[kk].gate)) return e;
        }
        while (k < all.size() && refs[k].round == r) ++k;
        for (int mm = 0; mm < 4; ++mm) {
            const auto &tl = tasks[r * 4 + mm];
            if (tl.empty()) continue;
            hipError_t e = qs::launch_tile_multi(10 + mm, uint32_t(tl.size()), dtasks + task_off[r * 4 + mm], dargs,
                                                 dops, dev + o_data, k5, nullptr, s->stream);
            if (e != hipSuccess) return hip_fail(e, "batched tile launch");
            ++B.st.launches;
        }
    }
    return QS_OK;
}

// Run sums (qs_traj.hip) of several trajectories, read back: sums[i]
// receives kRunMax + 1 doubles: Z, S_0, S_1, ...
qs_status batch_run_sums(Batch &B, const std::vector<int> &who, const std::vector<std::vector<int>> &qs_,
                         const std::vector<std::vector<double>> &as_, std::vector<std::vector<double>> &sums)
{
    qs_state *s = B.master;
    const uint64_t chunk = 1u << 16;
    std::vector<qs::RunSumArgs> args(who.size());
    std::vector<qs::RunSumTask> tasks;
    std::vector<uint32_t> first(who.size()), count(who.size());
    for (size_t i = 0; i < who.size(); ++i) {
        const int t = who[i];
        qs::RunSumArgs &a = args[i];
        a.amp = B.amp[t];
        a.n_amp = uint64_t(1) << B.prep[t].n;
        a.chunk_len = chunk;
        a.J = int(qs_[i].size());
        for (int j = 0; j < a.J; ++j) {
            a.q[j] = uint8_t(qs_[i][j]);
            a.am1[j] = as_[i][j] - 1.0;
        }
        const uint32_t nch = uint32_t((a.n_amp + chunk - 1) / chunk);
        first[i] = uint32_t(tasks.size());
        count[i] = nch;
        for (uint32_t c = 0; c < nch; ++c) tasks.push_back({uint32_t(i), c});
    }
    const int w = qs::kRunMax + 1;
    const size_t ab = align256(args.size() * sizeof(qs::RunSumArgs)), tb = align256(tasks.size() * sizeof(qs::RunSumTask));
    const size_t fb = align256(who.size() * 4);
    const size_t pb = align256(tasks.size() * w * sizeof(double)), ob = align256(who.size() * w * sizeof(double));
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(B.red.ensure(ab + tb + 2 * fb + pb + ob));
    unsigned char *dev = static_cast<unsigned char *>(B.red.p);
    HIP_TRY(hipMemcpy(dev, args.data(), args.size() * sizeof(qs::RunSumArgs), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dev + ab, tasks.data(), tasks.size() * sizeof(qs::RunSumTask), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dev + ab + tb, first.data(), who.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dev + ab + tb + fb, count.data(), who.size() * 4, hipMemcpyHostToDevice));
    double *partials = reinterpret_cast<double *>(dev + ab + tb + 2 * fb);
    double *out = reinterpret_cast<double *>(dev + ab + tb + 2 * fb + pb);
    {
        double bytes = 0;
        for (int t : who) bytes += double(amp_bytes(B.dt)) * std::ldexp(1.0, B.prep[t].n);
        Timed tm(s, QS_K_REDUCE, bytes, bytes);
        int nmax = 0;
        for (int t : who) nmax = std::max(nmax, B.prep[t].n);
        hipError_t e = qs::launch_run_sums(B.dt, nmax, uint32_t(tasks.size()), reinterpret_cast<qs::RunSumTask *>(dev + ab),
                                           reinterpret_cast<qs::RunSumArgs *>(dev), partials, nullptr, s->stream);
        if (e == hipSuccess)
            e = qs::launch_run_sums_finish(partials, reinterpret_cast<uint32_t *>(dev + ab + tb),
                                           reinterpret_cast<uint32_t *>(dev + ab + tb + fb), int(who.size()), out,
                                           s->stream);
        if (e != hipSuccess) return hip_fail(e, "trajectory reductions");
        B.st.launches += 2;
    }
    std::vector<double> host(who.size() * w);
    HIP_TRY(hipMemcpyAsync(host.data(), out, host.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    sums.assign(who.size(), {});
    for (size_t i = 0; i < who.size(); ++i) sums[i].assign(host.begin() + i * w, host.begin() + (i + 1) * w);
    return QS_OK;
}

// Branch choice of a RUN step from its sums (the same arithmetic as the
// device sampler): returns the first site that takes K2 and its weight, or
// -1 when every site takes K1.
int sample_run_host(const TStep &run, const std::vector<double> &sums, uint64_t seed, uint64_t traj, double &nrm2,
                    qs_status &err)
{
    err = QS_OK;
    double Z = sums[0];
    for (size_t j = 0; j < run.sites.size(); ++j) {
        const RunSite &rs = run.sites[j];
        const double c = -(rs.a - 1.0);
        const double cs = c * sums[1 + j];
        const double p2 = cs / Z;
        const double p1 = (Z - cs) / Z;
        const double u = qs::noise_uniform(seed, traj, rs.site);
        const int b = pick_branch({p1, p2}, u);
        if (b == 0) {
            Z -= cs;
            continue;
        }
        if (b < 0) {
            err = fail(QS_E_ZERO_NORM, "every Kraus branch has probability 0");
            return -1;
        }
        nrm2 = cs;
        return int(j);
    }
    return -1;
}

// <Z_q> of every listed trajectory from one batched pass of sums (a = 1).
qs_status host_expect_z(Batch &B, const std::vector<int> &who)
{
    if (who.empty()) return QS_OK;
    std::vector<std::vector<int>> qv(who.size());
    std::vector<std::vector<double>> av(who.size());
    for (size_t i = 0; i < who.size(); ++i)
        for (int q = 0; q < B.prep[who[i]].n; ++q) {
            qv[i].push_back(q);
            av[i].push_back(1.0);
        }
    std::vector<std::vector<double>> sums;
    if (qs_status e = batch_run_sums(B, who, qv, av, sums)) return e;
    for (size_t i = 0; i < who.size(); ++i) {
        const int t = who[i];
        const double Z = sums[i][0];
        for (int q = 0; q < B.prep[t].n; ++q) B.z_out[B.zoff[t] + q] = (Z - 2.0 * sums[i][1 + q]) / Z;
    }
    return QS_OK;
}

// Host-sampled path: all listed trajectories advance one step at a time.
qs_status run_host_sampled(Batch &B, const std::vector<int> &set)
{
    for (;;) {
        std::vector<int> gate_who, run_who;
        for (int t : set) {
            const TPrep &tp = B.prep[t];
            if (tp.cur >= tp.steps.size()) continue;
            (tp.steps[tp.cur].run ? run_who : gate_who).push_back(t);
        }
        if (gate_who.empty() && run_who.empty()) break;
        if (!gate_who.empty()) {
            std::vector<const std::vector<qs::FlatOp> *> lists;
            for (int t : gate_who) lists.push_back(&B.prep[t].steps[B.prep[t].cur].gates);
            if (qs_status e = batch_gates(B, gate_who, lists)) return e;
            for (int t : gate_who) ++B.prep[t].cur;
            continue;  // runs wait for the gates that precede them
        }
        std::vector<std::vector<int>> qv;
        std::vector<std::vector<double>> av;
        for (int t : run_who) {
            const TStep &r = B.prep[t].steps[B.prep[t].cur];
            qv.emplace_back();
            av.emplace_back();
            for (auto &s2 : r.sites) {
                qv.back().push_back(s2.q);
                av.back().push_back(s2.a);
            }
        }
        std::vector<std::vector<double>> sums;
        if (qs_status e = batch_run_sums(B, run_who, qv, av, sums)) return e;
        for (size_t i = 0; i < run_who.size(); ++i) {
            const int t = run_who[i];
            TPrep &tp = B.prep[t];
            double nrm2 = 0;
            qs_status err;
            const int j = sample_run_host(tp.steps[tp.cur], sums[i], B.seed, uint64_t(t), nrm2, err);
            if (err) return err;
            if (j < 0) {
                ++tp.cur;
            } else {
                jump_continuation(tp, tp.cur, size_t(j), nrm2);
                ++B.st.jumps;
            }
        }
    }
    return host_expect_z(B, set);
}

// ---------------------------------------------------- device-sampled path --

// Launch one pass job over the trajectories `job` (complex64 states of
// >= 10 qubits) in slot P: every remaining step planned, one upload, one
// graph (or the same launches enqueued directly) and the read-back of its
// results, all enqueued on the batch's stream; finish_pass reads them.
qs_status launch_pass(Batch &B, PassSlot &P, std::vector<int> job)
{
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    P.set = std::move(job);
    const std::vector<int> &set = P.set;
    const int S = int(set.size());
    const int w = qs::kRunMax + 1;
    qs_state *s = B.master;
    // ---- schedule: the rounds the host-sampled loop would run if no site jumped
    struct Ent { int slot; size_t step; };
    struct Round { bool run; std::vector<Ent> e; };
    std::vector<Round> rounds;
    {
        std::vector<size_t> cur(S);
        for (int i = 0; i < S; ++i) cur[i] = B.prep[set[i]].cur;
        for (;;) {
            Round g{false, {}}, r{true, {}};
            for (int i = 0; i < S; ++i) {
                const TPrep &tp = B.prep[set[i]];
                if (cur[i] >= tp.steps.size()) continue;
                (tp.steps[cur[i]].run ? r : g).e.push_back({i, cur[i]});
            }
            Round &take = g.e.empty() ? r : g;
            if (take.e.empty()) break;
            for (auto &e : take.e) ++cur[e.slot];
            rounds.push_back(std::move(take));
        }
    }
    // ---- plan every gate step, all in parallel
    struct PlanEnt { size_t round; int slot; size_t step; std::vector<qs::PlanStep> plan; };
    std::vector<PlanEnt> pe;
    for (size_t r = 0; r < rounds.size(); ++r)
        if (!rounds[r].run)
            for (auto &e : rounds[r].e) pe.push_back({r, e.slot, e.step, {}});
    parallel_for(pe.size(), [&](size_t k) {
        const TPrep &tp = B.prep[set[pe[k].slot]];
        plan_gate_list(B, tp.n, tp.steps[pe[k].step].gates, pe[k].plan);
    });
    P.out.assign(S, 0);  // plans with per-gate steps: host-sampled path instead
    std::vector<char> &out = P.out;
    for (auto &p : pe)
        for (auto &st : p.plan)
            if (!st.sweep) out[p.slot] = 1;
    // ---- launch list in round order; sweeps flattened in (round, sub-round, slot) order
    enum { L_TILE, L_RUN, L_FINAL };
    struct Launch {
        int kind = L_TILE;
        size_t a0 = 0, a1 = 0;      // L_TILE: sweeps [a0, a1) of one sub-round (expanded per tile width below)
        int m = 0;
        bool k5 = false;
        size_t t0 = 0, tn = 0;      // tile tasks / run-sum tasks
        size_t r0 = 0, rn = 0;      // run-sum args (rn = entries of the round)
        size_t fc0 = 0;             // first / count arrays (2 rn entries)
        size_t s0 = 0;              // sample args (rn entries)
        int nmax = 0;
    };
    std::vector<Launch> pre;
    std::vector<qs::PlanStep> all;
    std::vector<int> all_slot;
    std::vector<qs::RunSumArgs> rargs;
    std::vector<qs::RunSumTask> rtasks;
    std::vector<uint32_t> fc;
    std::vector<qs::SampleArgs> sargs;
    const uint64_t chunk = 1u << 16;
    size_t max_rtasks = 0, max_rows = 0;
    struct RunEnt { int slot; size_t step; const TStep *run; };  // run == NULL: final <Z> sums
    auto add_run_launch = [&](int kind, const std::vector<RunEnt> &ents) {
        Launch L;
        L.kind = kind;
        L.r0 = rargs.size();
        L.t0 = rtasks.size();
        L.fc0 = fc.size();
        L.s0 = sargs.size();
        L.rn = ents.size();
        fc.resize(fc.size() + 2 * ents.size());
        for (size_t i = 0; i < ents.size(); ++i) {
            const int slot = ents[i].slot;
            const int t = set[slot];
            const TPrep &tp = B.prep[t];
            qs::RunSumArgs a{};
            a.amp = B.amp[t];
            a.n_amp = uint64_t(1) << tp.n;
            a.chunk_len = chunk;
            a.slot = uint32_t(slot);
            if (kind == L_RUN) {
                const TStep &R = *ents[i].run;
                a.J = int(R.sites.size());
                qs::SampleArgs sa{};
                sa.slot = uint32_t(slot);
                sa.row = uint32_t(i);
                sa.traj = uint64_t(t);
                sa.step = uint32_t(ents[i].step);
                sa.arg = uint32_t(rargs.size());
                for (int j = 0; j < a.J; ++j) {
                    a.q[j] = uint8_t(R.sites[j].q);
                    a.am1[j] = R.sites[j].a - 1.0;
                    sa.site[j] = uint32_t(R.sites[j].site);
                }
                sargs.push_back(sa);
            } else {
                a.J = tp.n;
                for (int q = 0; q < tp.n; ++q) {
                    a.q[q] = uint8_t(q);
                    a.am1[q] = 0.0;
                }
            }
            const uint32_t nch = uint32_t((a.n_amp + chunk - 1) / chunk);
            fc[L.fc0 + i] = uint32_t(rtasks.size() - L.t0);
            fc[L.fc0 + ents.size() + i] = nch;
            for (uint32_t c = 0; c < nch; ++c) rtasks.push_back({uint32_t(rargs.size()), c});
            rargs.push_back(a);
            L.nmax = std::max(L.nmax, tp.n);
        }
        L.tn = rtasks.size() - L.t0;
        max_rtasks = std::max(max_rtasks, L.tn);
        max_rows = std::max(max_rows, L.rn);
        pre.push_back(L);
    };
    {
        size_t p = 0;
        for (size_t r = 0; r < rounds.size(); ++r) {
            if (!rounds[r].run) {
                size_t e = p;
                while (e < pe.size() && pe[e].round == r) ++e;
                size_t sub = 0;
                for (size_t i = p; i < e; ++i)
                    if (!out[pe[i].slot]) sub = std::max(sub, pe[i].plan.size());
                for (size_t k = 0; k < sub; ++k) {
                    Launch L;
                    L.kind = L_TILE;
                    L.a0 = all.size();
                    for (size_t i = p; i < e; ++i)
                        if (!out[pe[i].slot] && k < pe[i].plan.size()) {
                            all.push_back(std::move(pe[i].plan[k]));
                            all_slot.push_back(pe[i].slot);
                        }
                    L.a1 = all.size();
                    pre.push_back(L);
                }
                p = e;
                continue;
            }
            std::vector<RunEnt> ents;
            for (auto &e : rounds[r].e)
                if (!out[e.slot]) ents.push_back({e.slot, e.step, &B.prep[set[e.slot]].steps[e.step]});
            if (!ents.empty()) add_run_launch(L_RUN, ents);
        }
        std::vector<RunEnt> fin;
        for (int i = 0; i < S; ++i)
            if (!out[i]) fin.push_back({i, 0, nullptr});
        if (!fin.empty()) add_run_launch(L_FINAL, fin);
    }
    TileProgram tp;
    if (!all.empty()) build_tile_program(all, tp);
    std::vector<qs::TileArgsDev> targs(all.size());
    std::vector<qs::TileTask> ttasks;
    std::vector<Launch> L;
    for (const Launch &pl : pre) {
        if (pl.kind != L_TILE) {
            L.push_back(pl);
            continue;
        }
        for (size_t k = pl.a0; k < pl.a1; ++k) {
            const int t = set[all_slot[k]];
            qs::TileArgsDev &ad = targs[k];
            ad.amp = static_cast<float2 *>(B.amp[t]);
            ad.op_off = uint32_t(tp.first[k]);
            ad.slot = uint32_t(all_slot[k]);
            ad.ta = make_tile_args(all[k].sw, B.prep[t].n);
        }
        for (int m = 10; m <= 13; ++m) {
            Launch tl;
            tl.kind = L_TILE;
            tl.m = m;
            tl.t0 = ttasks.size();
            for (size_t k = pl.a0; k < pl.a1; ++k) {
                if (targs[k].ta.m != m) continue;
                for (size_t o = 0; o < all[k].sw.ops.size(); ++o) {
                    const qs::TileOpDev &d = tp.ops[tp.first[k] + o];
                    tl.k5 = tl.k5 || (d.kind == 0 && d.k == 5);
                }
                const uint32_t ntiles = uint32_t(1) << (B.prep[set[all_slot[k]]].n - m);
                for (uint32_t tile = 0; tile < ntiles; ++tile) ttasks.push_back({uint32_t(k), tile});
            }
            tl.tn = ttasks.size() - tl.t0;
            if (tl.tn) L.push_back(tl);
        }
    }
    // ---- one upload: program, arguments, tasks, activity flags, freeze records
    const size_t b_ops = tp.ops.size() * sizeof(qs::TileOpDev), b_data = tp.bytes();
    const size_t o_data = align256(b_ops);
    const size_t o_targs = o_data + align256(b_data);
    const size_t o_ttasks = o_targs + align256(targs.size() * sizeof(qs::TileArgsDev));
    const size_t o_rargs = o_ttasks + align256(ttasks.size() * sizeof(qs::TileTask));
    const size_t o_rtasks = o_rargs + align256(rargs.size() * sizeof(qs::RunSumArgs));
    const size_t o_fc = o_rtasks + align256(rtasks.size() * sizeof(qs::RunSumTask));
    const size_t o_sargs = o_fc + align256(fc.size() * sizeof(uint32_t));
    const size_t o_active = o_sargs + align256(sargs.size() * sizeof(qs::SampleArgs));
    const size_t o_freeze = o_active + align256(size_t(S) * sizeof(int));
    const size_t o_err = o_freeze + align256(size_t(S) * sizeof(qs::Freeze));
    const size_t up_bytes = o_err + 256;
    // device-only work space: partials, sums of one run round, final sums
    const size_t o_part = 0;
    const size_t o_sums = o_part + align256(std::max<size_t>(max_rtasks, 1) * w * sizeof(double));
    const size_t o_zs = o_sums + align256(std::max<size_t>(max_rows, 1) * w * sizeof(double));
    const size_t work_bytes = o_zs + align256(size_t(S) * w * sizeof(double));
    // the slot's previous job has been read (finish_pass), so its staging
    // and device buffers are free; a larger job regrows them, which waits
    // for the stream (the other slot's job may still run on it)
    {
        const size_t back_bytes = o_err - o_freeze + 256 + size_t(S) * w * sizeof(double);
        if (up_bytes > P.prog.cap || work_bytes > P.work.cap) HIP_TRY(hipStreamSynchronize(s->stream));
        if (up_bytes > P.prog.cap || work_bytes > P.work.cap || up_bytes > P.stage.cap || back_bytes > P.back.cap)
            B.grew = true;
        hipError_t e = P.prog.ensure(up_bytes);
        if (e == hipSuccess) e = P.work.ensure(work_bytes);
        if (e == hipSuccess) e = P.stage.ensure(up_bytes);
        if (e == hipSuccess) e = P.back.ensure(back_bytes);
        if (e == hipSuccess && !P.ev0) e = hipEventCreate(&P.ev0);
        if (e == hipSuccess && !P.ev1) e = hipEventCreate(&P.ev1);
        if (e == hipSuccess && !P.done) e = hipEventCreateWithFlags(&P.done, hipEventDisableTiming);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(QS_E_NOMEM, "trajectory pass buffers")
                                                               : hip_fail(e, "trajectory pass buffers");
    }
    unsigned char *host = static_cast<unsigned char *>(P.stage.p);
    struct Piece { size_t off; const void *src; size_t bytes; };
    std::vector<Piece> pieces = {{0, tp.ops.data(), b_ops},
                                 {o_targs, targs.data(), targs.size() * sizeof(qs::TileArgsDev)},
                                 {o_ttasks, ttasks.data(), ttasks.size() * sizeof(qs::TileTask)},
                                 {o_rargs, rargs.data(), rargs.size() * sizeof(qs::RunSumArgs)},
                                 {o_rtasks, rtasks.data(), rtasks.size() * sizeof(qs::RunSumTask)},
                                 {o_fc, fc.data(), fc.size() * sizeof(uint32_t)},
                                 {o_sargs, sargs.data(), sargs.size() * sizeof(qs::SampleArgs)}};
    parallel_for(pieces.size(), [&](size_t i) {
        if (pieces[i].bytes) std::memcpy(host + pieces[i].off, pieces[i].src, pieces[i].bytes);
    });
    if (b_data) tp.write(reinterpret_cast<uint16_t *>(host + o_data));
    {
        int *act = reinterpret_cast<int *>(host + o_active);
        qs::Freeze *fr = reinterpret_cast<qs::Freeze *>(host + o_freeze);
        for (int i = 0; i < S; ++i) {
            act[i] = out[i] ? 0 : 1;
            fr[i] = qs::Freeze{-1, 0, 0.0};
        }
        *reinterpret_cast<int *>(host + o_err) = 0;
    }
    unsigned char *dev = static_cast<unsigned char *>(P.prog.p);
    unsigned char *wk = static_cast<unsigned char *>(P.work.p);
    HIP_TRY(hipMemcpyAsync(dev, host, up_bytes, hipMemcpyHostToDevice, s->stream));
    const auto t1 = clock::now();
    // ---- the pass's launches
    const qs::TileOpDev *dops = reinterpret_cast<const qs::TileOpDev *>(dev);
    const qs::TileArgsDev *dtargs = reinterpret_cast<const qs::TileArgsDev *>(dev + o_targs);
    const qs::TileTask *dttasks = reinterpret_cast<const qs::TileTask *>(dev + o_ttasks);
    const qs::RunSumArgs *drargs = reinterpret_cast<const qs::RunSumArgs *>(dev + o_rargs);
    const qs::RunSumTask *drtasks = reinterpret_cast<const qs::RunSumTask *>(dev + o_rtasks);
    const uint32_t *dfc = reinterpret_cast<const uint32_t *>(dev + o_fc);
    const qs::SampleArgs *dsargs = reinterpret_cast<const qs::SampleArgs *>(dev + o_sargs);
    int *dactive = reinterpret_cast<int *>(dev + o_active);
    qs::Freeze *dfreeze = reinterpret_cast<qs::Freeze *>(dev + o_freeze);
    int *derr = reinterpret_cast<int *>(dev + o_err);
    double *dpart = reinterpret_cast<double *>(wk + o_part);
    double *dsums = reinterpret_cast<double *>(wk + o_sums);
    double *dzs = reinterpret_cast<double *>(wk + o_zs);
    int64_t nl = 0;
    auto enqueue = [&]() -> hipError_t {
        for (const Launch &l : L) {
            hipError_t e = hipSuccess;
            if (l.kind == L_TILE) {
                e = qs::launch_tile_multi(l.m, uint32_t(l.tn), dttasks + l.t0, dtargs, dops, dev + o_data, l.k5,
                                          dactive, s->stream);
                ++nl;
            } else {
                double *rows = l.kind == L_RUN ? dsums : dzs;
                e = qs::launch_run_sums(B.dt, l.nmax, uint32_t(l.tn), drtasks + l.t0, drargs, dpart, dactive,
                                        s->stream);
                if (e == hipSuccess)
                    e = qs::launch_run_sums_finish(dpart, dfc + l.fc0, dfc + l.fc0 + l.rn, int(l.rn), rows, s->stream);
                if (e == hipSuccess && l.kind == L_RUN)
                    e = qs::launch_sample_runs(dsargs + l.s0, uint32_t(l.rn), drargs, dsums, B.seed, dactive, dfreeze,
                                               derr, s->stream);
                nl += l.kind == L_RUN ? 3 : 2;
            }
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = hipEventRecord(P.ev0, s->stream);
    if (e == hipSuccess) {
        if (B.graph) {
            e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t el = enqueue();
                e = hipStreamEndCapture(s->stream, &P.graph);
                if (el != hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0);
            if (e == hipSuccess) e = hipGraphLaunch(P.exec, s->stream);
        } else {
            e = enqueue();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(P.ev1, s->stream);
    unsigned char *back = static_cast<unsigned char *>(P.back.p);
    P.zb = o_err - o_freeze + 256;
    P.err_at = o_err - o_freeze;
    if (e == hipSuccess) e = hipMemcpyAsync(back, dev + o_freeze, P.zb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(back + P.zb, dzs, size_t(S) * w * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipEventRecord(P.done, s->stream);
    if (e != hipSuccess) {
        P.drop_graph();
        return hip_fail(e, "trajectory pass");
    }
    P.busy = true;
    // the job's plans and operand pieces are many small allocations: freed
    // in parallel (on one thread, as the locals go out of scope, about 5 ms
    // per job of 64 trajectories, while the device waits for the next job)
    parallel_for(all.size(), [&](size_t i) { all[i] = qs::PlanStep(); });
    parallel_for(tp.piece.size(), [&](size_t i) { std::vector<uint16_t>().swap(tp.piece[i]); });
    B.st.host_seconds += std::chrono::duration<double>(t1 - t0).count();
    B.st.launches += nl;
    ++B.st.graphs;
    return QS_OK;
}

// Wait for slot P's job and read its results: completed trajectories write
// <Z_q>; those whose run took K2 are rewritten from the jump on and go to
// `next`; those whose plans need per-gate launches go to `demoted`.
qs_status finish_pass(Batch &B, PassSlot &P, std::vector<int> &next, std::vector<int> &demoted)
{
    const int w = qs::kRunMax + 1;
    P.busy = false;
    hipError_t e = hipEventSynchronize(P.done);
    P.drop_graph();
    if (e != hipSuccess) return hip_fail(e, "trajectory pass");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.ev0, P.ev1) == hipSuccess) B.st.device_seconds += 1e-3 * ms;
    const unsigned char *back = static_cast<const unsigned char *>(P.back.p);
    if (*reinterpret_cast<const int *>(back + P.err_at))
        return fail(QS_E_ZERO_NORM, "every Kraus branch of a damping site has probability 0");
    const qs::Freeze *fr = reinterpret_cast<const qs::Freeze *>(back);
    const double *zs = reinterpret_cast<const double *>(back + P.zb);
    size_t row = 0;
    for (size_t i = 0; i < P.set.size(); ++i) {
        const int t = P.set[i];
        if (P.out[i]) {
            demoted.push_back(t);
            continue;
        }
        TPrep &tp = B.prep[t];
        const double *z = zs + row * w;
        ++row;
        if (fr[i].step < 0) {
            const double Z = z[0];
            for (int q = 0; q < tp.n; ++q) B.z_out[B.zoff[t] + q] = (Z - 2.0 * z[1 + q]) / Z;
            tp.cur = tp.steps.size();
            continue;
        }
        jump_continuation(tp, size_t(fr[i].step), size_t(fr[i].j), fr[i].nrm2);
        ++B.st.jumps;
        next.push_back(t);
    }
    return QS_OK;
}

// Device-sampled jobs over `set` until no trajectory is left.  Trajectories
// wait in `pending`, in order; a job takes up to B.par.chunk of them.  Jobs
// go alternately to two slots, so that the host builds a job while the device
// runs the one before it; before a slot is reused its previous job is
// finished, and that job's trajectories that jumped join `pending` at once:
// they run in the next job instead of after the rest of the batch.  The
// passes reported are the most jobs any one trajectory ran in.
qs_status run_device_sampled(Batch &B, std::vector<int> set, std::vector<int> &demoted)
{
    const size_t C = B.par.chunk > 0 ? size_t(B.par.chunk) : std::max<size_t>(set.size(), 1);
    std::vector<int> pending(std::move(set)), runs(B.prep.size(), 0);
    size_t head = 0;
    int passes = 0;
    auto finish = [&](PassSlot &P) -> qs_status {
        std::vector<int> next;
        if (qs_status e = finish_pass(B, P, next, demoted)) return e;
        pending.insert(pending.end(), next.begin(), next.end());
        return QS_OK;
    };
    for (int k = 0;; ++k) {
        PassSlot &P = B.slot[k & 1], &O = B.slot[(k + 1) & 1];  // P holds the older job
        if (P.busy)
            if (qs_status e = finish(P)) return e;
        if (head == pending.size()) {  // nothing waiting: the newer job may still add some
            if (!O.busy) break;
            if (qs_status e = finish(O)) return e;
            if (head == pending.size()) break;
        }
        const size_t take = std::min(C, pending.size() - head);
        std::vector<int> job(pending.begin() + long(head), pending.begin() + long(head + take));
        head += take;
        for (int t : job) passes = std::max(passes, ++runs[size_t(t)]);
        if (qs_status e = prepare_some(B, job)) return e;
        if (qs_status e = launch_pass(B, P, std::move(job))) return e;
    }
    B.st.passes += passes;
    return QS_OK;
}

qs_status run_trajectory_batch(const qs_circuit *const *circs, const int *widths, int count, qs_dtype dt,
                               uint64_t seed, const TrajParams &par, bool device_ok, bool graph, double *z_out,
                               qs_traj_stats &stats, bool &cold)
{
    cold = false;
    if (!circs || !widths || !z_out || count < 0) return fail(QS_E_INVAL, "NULL argument or negative count");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", int(dt));
    if (count == 0) return QS_OK;
    const auto t0 = std::chrono::steady_clock::now();
    Batch B;
    B.dt = dt;
    B.par = par;
    B.graph = graph;
    B.seed = seed;
    B.z_out = z_out;
    B.circs = circs;
    B.widths = widths;
    B.prep.resize(count);
    B.ready.assign(size_t(count), 0);
    size_t total = 0;
    for (int t = 0; t < count; ++t) {
        if (!circs[t]) return fail(QS_E_INVAL, "circuit %d is NULL", t);
        if (widths[t] < 1 || widths[t] > qs::kRunMax) return fail(QS_E_INVAL, "width %d not in [1, %d]", widths[t], qs::kRunMax);
        total += amp_bytes(dt) << widths[t];
        B.prep[t].n = widths[t];  // the rest when its job is built (prepare_some)
    }
    const size_t lim = g_mem_limit.load();
    if (lim && total > lim) return fail(QS_E_NOMEM, "batch of %zu bytes exceeds the memory limit", total);
    if (qs_status e = qs_create(1, dt, &B.master)) return e;
    HIP_TRY(hipGetDevice(&B.dev));
    B.slot = take_slots(B.dev);
    {
        hipError_t e = B.states.ensure(total);
        if (e != hipSuccess) return fail(QS_E_NOMEM, "device allocation of %zu bytes failed", total);
    }
    size_t off = 0, zo = 0;
    for (int t = 0; t < count; ++t) {
        B.amp.push_back(static_cast<unsigned char *>(B.states.p) + off);
        B.views.push_back(new View(B.master, B.amp.back(), widths[t]));
        B.zoff.push_back(zo);
        off += amp_bytes(dt) << widths[t];
        zo += size_t(widths[t]);
    }
    for (int t = 0; t < count; ++t)
        if (qs_status e = init_amplitudes(&B.views[t]->s)) return e;
    std::vector<int> dev_set, host_set;
    for (int t = 0; t < count; ++t) (device_ok && device_sampled(B, t) ? dev_set : host_set).push_back(t);
    B.st.graph = graph && !dev_set.empty();
    {
        std::vector<int> demoted;
        if (qs_status e = run_device_sampled(B, dev_set, demoted)) return e;
        host_set.insert(host_set.end(), demoted.begin(), demoted.end());
    }
    B.st.host_sampled = int(host_set.size());
    if (qs_status e = prepare_some(B, host_set)) return e;
    if (qs_status e = run_host_sampled(B, host_set)) return e;
    HIP_TRY(hipStreamSynchronize(B.master->stream));
    B.st.tile_qubits = par.m_cap;
    B.st.k_max = par.kmax;
    B.st.max_outer = par.max_outer;
    B.st.chunk = par.chunk;
    B.st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats = B.st;
    cold = B.grew;
    return QS_OK;
}

}  // namespace

namespace {

qs_status check_mlp(const float *params, int f, int h)
{
    if (!params) return fail(QS_E_INVAL, "params is NULL");
    if (f < 1 || f > 256) return fail(QS_E_INVAL, "feature count %d not in [1, 256]", f);
    if (h != qs::kMlpHidden) return fail(QS_E_UNSUPPORTED, "hidden width must be %d", qs::kMlpHidden);
    return QS_OK;
}

struct DevTmp {
    std::vector<void *> p;
    ~DevTmp()
    {
        for (void *q : p) (void)hipFree(q);
    }
    template <typename T>
    hipError_t alloc(T **out, size_t count)
    {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, count * sizeof(T) + 16);
        if (e == hipSuccess) p.push_back(q);
        *out = static_cast<T *>(q);
        return e;
    }
};

}  // namespace

// =================================================================== ABI ==

extern "C" {

const char *qs_last_error(void) { return g_err; }

qs_status qs_set_memory_limit(size_t bytes)
try {
    g_mem_limit.store(bytes);
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_create(int n, qs_dtype dt, qs_state **out)
try {
    qs_status st = create_common(n, dt, out);
    if (st) return st;
    const size_t bytes = amp_bytes(dt) << n;
    const size_t lim = g_mem_limit.load();
    if (lim && bytes > lim)
        return fail(QS_E_NOMEM, "state of %zu bytes exceeds the memory limit of %zu bytes", bytes, lim);
    qs_state *s = new (std::nothrow) qs_state();
    if (!s) return fail(QS_E_NOMEM, "host allocation failed");
    s->n = n;
    s->dt = dt;
    s->bytes = bytes;
    hipGetDevice(&s->device);
    hipError_t e = hipMalloc(&s->amp, bytes);
    if (e != hipSuccess) {
        s->amp = nullptr;
        free_state(s);
        hipGetLastError();
        return fail(QS_E_NOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_state(s);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    s->own_stream = true;
    if ((st = alloc_state_buffers(s)) || (st = init_amplitudes(s))) {
        free_state(s);
        return st;
    }
    *out = s;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_create_from_buffer(int n, qs_dtype dt, void *buf, size_t bytes, void *stream,
                                qs_state **out)
try {
    qs_status st = create_common(n, dt, out);
    if (st) return st;
    if (!buf) return fail(QS_E_INVAL, "device buffer is NULL");
    const size_t need = amp_bytes(dt) << n;
    if (bytes < need) return fail(QS_E_INVAL, "buffer of %zu bytes, %zu needed", bytes, need);
    if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(QS_E_INVAL, "buffer is not 16-byte aligned");
    qs_state *s = new (std::nothrow) qs_state();
    if (!s) return fail(QS_E_NOMEM, "host allocation failed");
    s->n = n;
    s->dt = dt;
    s->bytes = need;
    s->amp = buf;
    s->owned = false;
    s->stream = (hipStream_t)stream;
    hipGetDevice(&s->device);
    if ((st = alloc_state_buffers(s)) || (st = init_amplitudes(s))) {
        free_state(s);
        return st;
    }
    *out = s;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_destroy(qs_state *s)
try {
    free_state(s);
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_reset(qs_state *s)
try {
    if (qs_status st = check_state(s)) return st;
    return init_amplitudes(s);
} QS_ABI_CATCH

qs_status qs_set_amplitudes(qs_state *s, const double *amps)
try {
    if (qs_status st = check_state(s)) return st;
    if (!amps) return fail(QS_E_INVAL, "amplitudes are NULL");
    const size_t na = size_t(1) << s->n;
    if (s->dt == QS_C128) {
        HIP_TRY(hipMemcpyAsync(s->amp, amps, na * 16, hipMemcpyHostToDevice, s->stream));
    } else {
        std::vector<float> f(2 * na);
        for (size_t k = 0; k < 2 * na; ++k) f[k] = float(amps[k]);
        HIP_TRY(hipMemcpyAsync(s->amp, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_info(const qs_state *s, int *n, qs_dtype *dt, void **dev, void **stream)
try {
    if (qs_status st = check_state(s)) return st;
    if (n) *n = s->n;
    if (dt) *dt = s->dt;
    if (dev) *dev = s->amp;
    if (stream) *stream = (void *)s->stream;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_synchronize(qs_state *s)
try {
    if (qs_status st = check_state(s)) return st;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_apply_gate(qs_state *s, const int *targets, int nt, const int *controls, int nc,
                        const double *m)
try {
    if (qs_status st = check_state(s)) return st;
    if (qs_status st = check_qubits(s->n, targets, nt, controls, nc, QS_MAX_TARGETS)) return st;
    if (qs_status st = check_matrix(m, nt)) return st;
    return apply_gate_host(s, targets, nt, controls, nc, m);
} QS_ABI_CATCH

qs_status qs_apply_noisy_gate(qs_state *s, const int *targets, int nt, const int *controls, int nc,
                              const double *m, const double *kraus, int nk, double u, int *chosen,
                              double *p_chosen)
try {
    if (qs_status st = check_state(s)) return st;
    if (nc != 0) return fail(QS_E_UNSUPPORTED, "noisy gates with controls are not supported");
    if (qs_status st = check_qubits(s->n, targets, nt, controls, 0, QS_MAX_TARGETS)) return st;
    if (qs_status st = check_matrix(m, nt)) return st;
    if (qs_status st = check_kraus(kraus, nk, nt)) return st;
    if (!(u >= 0.0 && u < 1.0)) return fail(QS_E_INVAL, "u = %g not in [0, 1)", u);
    if (qs_status st = apply_gate_host(s, targets, nt, nullptr, 0, m)) return st;
    return apply_channel(s, targets, nt, kraus, nk, u, chosen, p_chosen);
} QS_ABI_CATCH

// ------------------------------------------------------------- circuits --

qs_status qs_circuit_create(qs_circuit **out)
try {
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    *out = new (std::nothrow) qs_circuit();
    if (!*out) return fail(QS_E_NOMEM, "host allocation failed");
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_circuit_destroy(qs_circuit *c)
try {
    delete c;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_circuit_append_gate(qs_circuit *c, const int *targets, int nt, const int *controls,
                                 int nc, const double *m)
try {
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (qs_status st = check_qubits(QS_MAX_CIRCUIT_QUBITS, targets, nt, controls, nc, QS_MAX_TARGETS)) return st;
    if (qs_status st = check_matrix(m, nt)) return st;
    qs::Op op;
    op.kind = qs::Op::GATE;
    op.targets.assign(targets, targets + nt);
    if (nc) op.controls.assign(controls, controls + nc);
    op.m.assign(m, m + (size_t(2) << (2 * nt)));
    c->ops.push_back(std::move(op));
    c->changed();
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_circuit_append_noise(qs_circuit *c, const int *targets, int nt, const double *kraus, int nk)
try {
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (qs_status st = check_qubits(QS_MAX_CIRCUIT_QUBITS, targets, nt, nullptr, 0, QS_MAX_TARGETS)) return st;
    if (qs_status st = check_kraus(kraus, nk, nt)) return st;
    if (c->ops.empty() || c->ops.back().kind != qs::Op::GATE)
        return fail(QS_E_INVAL, "a noise site must follow a gate");
    const qs::Op &g = c->ops.back();
    if (!g.controls.empty() || g.targets != std::vector<int>(targets, targets + nt))
        return fail(QS_E_INVAL, "a noise site must have the targets of the gate before it and that gate no controls");
    qs::Op op;
    op.kind = qs::Op::NOISE;
    op.targets.assign(targets, targets + nt);
    op.nk = nk;
    op.m.assign(kraus, kraus + (size_t(2) << (2 * nt)) * nk);
    c->ops.push_back(std::move(op));
    c->changed();
    return QS_OK;
} QS_ABI_CATCH

static qs_status push_marker(qs_circuit *c, qs::Op::Kind k, int q)
{
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (k == qs::Op::BEGIN_CONTROL && (q < 0 || q >= QS_MAX_CIRCUIT_QUBITS))
        return fail(QS_E_RANGE, "control qubit %d out of range", q);
    qs::Op op;
    op.kind = k;
    op.qubit = q;
    c->ops.push_back(std::move(op));
    c->changed();
    return QS_OK;
}

qs_status qs_circuit_begin_dagger(qs_circuit *c) try { return push_marker(c, qs::Op::BEGIN_DAGGER, -1); } QS_ABI_CATCH
qs_status qs_circuit_end_dagger(qs_circuit *c) try { return push_marker(c, qs::Op::END_DAGGER, -1); } QS_ABI_CATCH
qs_status qs_circuit_begin_control(qs_circuit *c, int q) try { return push_marker(c, qs::Op::BEGIN_CONTROL, q); } QS_ABI_CATCH
qs_status qs_circuit_end_control(qs_circuit *c) try { return push_marker(c, qs::Op::END_CONTROL, -1); } QS_ABI_CATCH

qs_status qs_circuit_counts(const qs_circuit *c, int64_t *gates, int64_t *noise, int64_t *logical)
try {
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    std::vector<qs::FlatOp> flat;
    std::string err;
    if (qs::expand(c->ops, flat, err)) return fail(QS_E_INVAL, "%s", err.c_str());
    int64_t g = 0, z = 0, l = 0;
    for (auto &f : flat) {
        if (f.kind == qs::FlatOp::GATE) {
            ++g;
            if (!qs::is_identity(f.m, int(f.targets.size()))) ++l;
        } else {
            ++z;
        }
    }
    if (gates) *gates = g;
    if (noise) *noise = z;
    if (logical) *logical = l;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_circuit_plan_info(const qs_circuit *c, int n, qs_dtype dt, const qs_run_opts *opts,
                               int64_t *sweeps, int64_t *blocks, int64_t *logical)
try {
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (n < 1 || n > QS_MAX_QUBITS) return fail(QS_E_INVAL, "n = %d not in [1, %d]", n, QS_MAX_QUBITS);
    qs_run_opts o{};
    if (opts) o = *opts;
    if (o.plan == QS_PLAN_AUTOTUNE) {
        // the fastest candidate measured so far, else the greedy defaults
        int tq = 0, km = 0;
        qs_circuit_autotune_result(c, n, dt, nullptr, nullptr, &tq, &km, nullptr);
        o.plan = QS_PLAN_GREEDY;
        o.tile_qubits = tq;
        o.k_max = km;
    }
    std::vector<qs::FlatOp> flat;
    std::string err;
    if (int rc = qs::expand(c->ops, flat, err)) return fail(rc == 2 ? QS_E_UNSUPPORTED : QS_E_INVAL, "%s", err.c_str());
    for (auto &f : flat) {
        for (int q : f.targets)
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        for (int q : f.controls)
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
    }
    int64_t sw = 0, bl = 0, lg = 0;
    qs_state probe;
    probe.n = n;
    probe.dt = dt;
    size_t k = 0;
    while (k < flat.size()) {
        size_t e = k;
        while (e < flat.size() && flat[e].kind == qs::FlatOp::GATE) {
            if (!qs::is_identity(flat[e].m, int(flat[e].targets.size()))) ++lg;
            ++e;
        }
        if (e > k) {
            if (tiled_plan(&probe, o)) {
                std::vector<qs::PlanStep> steps;
                qs::TileParams tp;
                if (qs_status st = choose_tile_params(&probe, flat, k, e, o, tp, steps)) return st;
                for (auto &st : steps) {
                    ++sw;
                    bl += st.sweep ? int64_t(st.sw.ops.size()) : 1;
                }
            } else {
                std::vector<qs::CanonGate> plan;
                if (o.plan == QS_PLAN_UNFUSED) {
                    for (size_t j = k; j < e; ++j)
                        plan.push_back(qs::canonicalize(flat[j].targets.data(), int(flat[j].targets.size()),
                                                        flat[j].controls.data(), int(flat[j].controls.size()),
                                                        flat[j].m.data()));
                } else {
                    qs::greedy_fuse(flat, k, e, o.k_max ? o.k_max : qs::default_kmax(n, dt), plan);
                }
                for (auto &g : plan)
                    if (g.kind != qs::CanonGate::IDENTITY) ++sw, ++bl;
            }
        }
        k = e < flat.size() ? e + 1 : e;
    }
    if (sweeps) *sweeps = sw;
    if (blocks) *blocks = bl;
    if (logical) *logical = lg;
    return QS_OK;
} QS_ABI_CATCH

}  // extern "C"

namespace {

// Candidate fused plans of a state shape for QS_PLAN_AUTOTUNE.
std::vector<Tuning::Cand> autotune_candidates(int n, qs_dtype dt)
{
    std::vector<Tuning::Cand> c;
    if (dt == QS_C64 && n >= 11) {
        for (int m = 11; m <= 13 && m <= n; ++m)
            for (int k = 4; k <= 5; ++k) c.push_back({m, k, -1.0});
    } else {
        for (int k = 2; k <= 4 && k <= n; ++k) c.push_back({0, k, -1.0});
    }
    return c;
}

qs_status plan_circuit(qs_state *s, const qs_circuit *c, const qs_run_opts &o,
                       std::shared_ptr<const CachedPlan> &cp);
qs_status execute_plan(qs_state *s, const CachedPlan &plan, qs_run_opts o);

// One run under QS_PLAN_AUTOTUNE: the next untried candidate, timed, or the
// fastest one.
qs_status run_autotuned(qs_state *s, const qs_circuit *c, qs_run_opts o)
{
    int cand = -1;
    Tuning::Cand pick{};
    {
        std::lock_guard<std::mutex> lk(c->mu);
        Tuning &t = c->tuning[{s->n, int(s->dt)}];
        if (t.cands.empty()) t.cands = autotune_candidates(s->n, s->dt);
        if (t.next < t.cands.size()) {
            cand = int(t.next++);
            pick = t.cands[cand];
        } else {
            pick = t.cands[t.best >= 0 ? t.best : 0];
        }
    }
    o.plan = QS_PLAN_GREEDY;
    o.k_max = pick.kmax;
    o.tile_qubits = pick.tile;
    std::shared_ptr<const CachedPlan> cp;
    if (qs_status st = plan_circuit(s, c, o, cp)) return st;
    if (cand < 0) return execute_plan(s, *cp, o);
    // operand programs of a single tiled segment go up before the clock starts
    size_t tiled = 0;
    const SegPlan *only = nullptr;
    for (const SegPlan &sp : cp->segs)
        if (sp.tiled) ++tiled, only = &sp;
    if (tiled == 1) {
        size_t doff = 0;
        if (qs_status st = upload_program(s, only->prog, only->prog_id, doff)) return st;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(QS_E_DEVICE, "hipEventCreate failed");
    }
    qs_status st = QS_OK;
    float ms = 0.f;
    if (hipEventRecord(e0, s->stream) != hipSuccess) st = fail(QS_E_DEVICE, "hipEventRecord failed");
    if (!st) st = execute_plan(s, *cp, o);
    if (!st && (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(QS_E_DEVICE, "timing the autotuning run failed");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    Tuning &t = c->tuning[{s->n, int(s->dt)}];
    if (size_t(cand) < t.cands.size()) {
        t.cands[cand].seconds = double(ms) * 1e-3;
        if (t.best < 0 || t.cands[cand].seconds < t.cands[t.best].seconds) t.best = cand;
    }
    return QS_OK;
}

}  // namespace

extern "C" {

qs_status qs_circuit_autotune_result(const qs_circuit *c, int n, qs_dtype dt, int *tried, int *candidates,
                                     int *tile_qubits, int *k_max, double *seconds)
try {
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (n < 1 || n > QS_MAX_QUBITS) return fail(QS_E_INVAL, "n = %d not in [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", int(dt));
    std::lock_guard<std::mutex> lk(c->mu);
    int tr = 0, nc = int(autotune_candidates(n, dt).size()), tq = 0, km = 0;
    double sec = 0.0;
    auto it = c->tuning.find({n, int(dt)});
    if (it != c->tuning.end()) {
        const Tuning &t = it->second;
        for (const auto &cd : t.cands) tr += cd.seconds >= 0.0;
        if (t.best >= 0) {
            tq = t.cands[t.best].tile;
            km = t.cands[t.best].kmax;
            sec = t.cands[t.best].seconds;
        }
    }
    if (tried) *tried = tr;
    if (candidates) *candidates = nc;
    if (tile_qubits) *tile_qubits = tq;
    if (k_max) *k_max = km;
    if (seconds) *seconds = sec;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_run_circuit(qs_state *s, const qs_circuit *c, const qs_run_opts *opts)
try {
    if (qs_status st = check_state(s)) return st;
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    qs_run_opts o{};
    if (opts) o = *opts;
    if (o.plan < QS_PLAN_UNFUSED || o.plan > QS_PLAN_AUTOTUNE) return fail(QS_E_INVAL, "unknown plan %d", o.plan);
    if (o.k_max < 0 || o.k_max > QS_MAX_TARGETS) return fail(QS_E_INVAL, "k_max = %d not in [0, %d]", o.k_max, QS_MAX_TARGETS);
    if (o.tile_qubits && (o.tile_qubits < 10 || o.tile_qubits > 13))
        return fail(QS_E_INVAL, "tile_qubits = %d not in [10, 13]", o.tile_qubits);
    if (o.tile_order < 0 || o.tile_order > QS_TILE_ORDERS)
        return fail(QS_E_INVAL, "tile_order = %d not in [0, %d]", o.tile_order, QS_TILE_ORDERS);
    if (o.plan == QS_PLAN_AUTOTUNE) return run_autotuned(s, c, o);
    std::shared_ptr<const CachedPlan> cp;
    if (qs_status st = plan_circuit(s, c, o, cp)) return st;
    return execute_plan(s, *cp, o);
} QS_ABI_CATCH

namespace {

// The cached plan of (state shape, options), made on first use.
qs_status plan_circuit(qs_state *s, const qs_circuit *c, const qs_run_opts &o,
                       std::shared_ptr<const CachedPlan> &cp)
{
    const PlanKey key{s->n, int(s->dt), o.plan, o.k_max, o.tile_qubits,
                      o.plan == QS_PLAN_LEARNED ? g_model_version.load() : 0};
    cp.reset();
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->cache.find(key);
        if (it != c->cache.end()) cp = it->second;
    }
    if (!cp) {
        std::vector<qs::FlatOp> flat;
        std::string err;
        int rc = qs::expand(c->ops, flat, err);
        if (rc == 2) return fail(QS_E_UNSUPPORTED, "%s", err.c_str());
        if (rc) return fail(QS_E_INVAL, "%s", err.c_str());
        for (auto &f : flat) {
            for (int q : f.targets)
                if (q >= s->n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, s->n);
            for (int q : f.controls)
                if (q >= s->n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, s->n);
        }
        auto np = std::make_shared<CachedPlan>();
        size_t k = 0;
        while (k < flat.size()) {
            // segment of gates up to the next noise site
            size_t e = k;
            while (e < flat.size() && flat[e].kind == qs::FlatOp::GATE) ++e;
            SegPlan sp;
            if (e > k) {
                if (tiled_plan(s, o)) {
                    sp.tiled = true;
                    qs::TileParams tp;
                    if (qs_status st = choose_tile_params(s, flat, k, e, o, tp, sp.steps)) return st;
                    build_tile_program(sp.steps, sp.prog);
                    sp.prog.materialize();
                    sp.prog_id = g_prog_serial.fetch_add(1);
                    sp.tune = std::make_shared<OrderTune>();
                } else if (o.plan == QS_PLAN_UNFUSED) {
                    for (size_t j = k; j < e; ++j)
                        sp.gates.push_back(qs::canonicalize(flat[j].targets.data(), int(flat[j].targets.size()),
                                                            flat[j].controls.data(), int(flat[j].controls.size()),
                                                            flat[j].m.data()));
                } else {
                    const int kmax = o.k_max ? o.k_max : qs::default_kmax(s->n, s->dt);
                    qs::greedy_fuse(flat, k, e, kmax, sp.gates);
                }
            }
            if (e < flat.size()) {
                sp.has_noise = true;
                sp.noise = flat[e];
                ++e;
            }
            np->segs.push_back(std::move(sp));
            k = e;
        }
        cp = np;
        std::lock_guard<std::mutex> lk(c->mu);
        c->cache[key] = cp;
    }
    return QS_OK;
}

qs_status execute_plan(qs_state *s, const CachedPlan &plan, qs_run_opts o)
{
    uint64_t site = 0;
    for (const SegPlan &sp : plan.segs) {
        if (sp.tiled) {
            if (qs_status st = launch_steps(s, sp.steps, sp.prog, sp.prog_id, sp.tune.get(), o.tile_order))
                return st;
        } else if (!sp.gates.empty()) {
            if (qs_status st = launch_plan(s, sp.gates)) return st;
        }
        if (sp.has_noise) {
            const qs::FlatOp &z = sp.noise;
            const double u = qs_philox_uniform(o.seed, o.traj, site);
            int ch = -1;
            if (qs_status st = apply_channel(s, z.targets.data(), int(z.targets.size()), z.m.data(), z.nk,
                                             u, &ch, nullptr))
                return st;
            if (o.chosen && int64_t(site) < o.chosen_len) o.chosen[site] = ch;
            ++site;
        }
    }
    return QS_OK;
}

}  // namespace

// ------------------------------------------------------- sharded states --

namespace {

qs_status remap(qs_state *s, int g, const int *lq, const void *buf, bool pack)
{
    if (qs_status st = check_state(s)) return st;
    const int L = s->n;
    if (g < 0 || g > L || g > QS_REMAP_MAX_G)
        return fail(QS_E_INVAL, "g = %d not in [0, %d]", g, L < QS_REMAP_MAX_G ? L : QS_REMAP_MAX_G);
    if (g > 0 && !lq) return fail(QS_E_INVAL, "lq is NULL");
    if (!buf) return fail(QS_E_INVAL, "device_buf is NULL");
    if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(QS_E_INVAL, "device_buf is not 16-byte aligned");
    uint64_t seen = 0;
    for (int i = 0; i < g; ++i) {
        if (lq[i] < 0 || lq[i] >= L) return fail(QS_E_RANGE, "local qubit %d not in [0, %d)", lq[i], L);
        if ((seen >> lq[i]) & 1) return fail(QS_E_RANGE, "local qubit %d repeated", lq[i]);
        seen |= uint64_t(1) << lq[i];
    }
    const size_t bytes = amp_bytes(s->dt) << L;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(buf), a0 = reinterpret_cast<uintptr_t>(s->amp);
    if (b0 < a0 + bytes && a0 < b0 + bytes) return fail(QS_E_INVAL, "device_buf overlaps the state");
    hipError_t e;
    {
        Timed t(s, QS_K_OTHER, 2.0 * double(bytes), 0.0);
        e = qs::launch_remap(s->dt, s->amp, const_cast<void *>(buf), L, g, lq, pack, s->stream);
    }
    if (e != hipSuccess) return hip_fail(e, pack ? "remap pack" : "remap unpack");
    return QS_OK;
}

}  // namespace

qs_status qs_remap_pack(const qs_state *s, int g, const int *lq, void *device_buf)
try {
    return remap(const_cast<qs_state *>(s), g, lq, device_buf, true);
} QS_ABI_CATCH

qs_status qs_remap_unpack(qs_state *s, int g, const int *lq, const void *device_buf)
try {
    return remap(s, g, lq, device_buf, false);
} QS_ABI_CATCH

// ------------------------------------------------ partial-amplitude mode --

namespace {

// Device memory up to which the partial mode keeps one state per level of
// the cut tree (partial_tree) instead of rerunning each branch word in full.
constexpr double kPartialTreeBytes = 32.0 * (1ull << 30);

// A gate of one part's sub-circuit, qubits in that part's numbering; the
// matrix in the ABI layout (2^nt x 2^nt, row-major (re, im) pairs).
struct PartGate {
    std::vector<int> t, c;
    std::vector<double> m;
};

// A crossing gate cut as in Eq. 4: on branch b, part `pside` receives the
// diagonal projector proj[b] and the other part other[b] (when has[b]).
struct PartCut {
    int pside = 0;
    PartGate proj[2], other[2];
    bool has[2] = {false, false};
};

struct PartialPlan {
    int n = 0, np[2] = {0, 0};
    std::vector<int> side, pos;            // qubit -> part (0 = A, 1 = B), index in the part
    std::vector<std::pair<int, PartGate>> items;  // (part, gate) or (2 + cut index, {})
    std::vector<PartCut> cuts;
};

qs_status build_partial(const qs_circuit *c, int n, uint64_t part_a, PartialPlan &pp)
{
    // diagonal gate on `qs_` (qs_[0] = most significant bit of the index)
    // with factors f(y), y < 2^|qs_|
    auto diag_gate = [](const std::vector<int> &qs_, const std::function<cd(uint32_t)> &f) {
        PartGate g;
        g.t = qs_;
        const size_t d = size_t(1) << qs_.size();
        g.m.assign(2 * d * d, 0.0);
        for (size_t y = 0; y < d; ++y) {
            const cd v = f(uint32_t(y));
            g.m[2 * (y * d + y)] = v.real();
            g.m[2 * (y * d + y) + 1] = v.imag();
        }
        return g;
    };
    if (!c) return fail(QS_E_INVAL, "circuit is NULL");
    if (n < 2 || n > 62) return fail(QS_E_INVAL, "n = %d not in [2, 62]", n);
    const uint64_t all = (uint64_t(1) << n) - 1;
    if (part_a & ~all) return fail(QS_E_INVAL, "part_a names qubits >= n = %d", n);
    pp = PartialPlan{};
    pp.n = n;
    pp.side.resize(n);
    pp.pos.resize(n);
    for (int q = 0; q < n; ++q) {
        pp.side[q] = (part_a >> q) & 1 ? 0 : 1;
        pp.pos[q] = pp.np[pp.side[q]]++;
    }
    for (int p = 0; p < 2; ++p)
        if (pp.np[p] < 1 || pp.np[p] > QS_MAX_QUBITS) {
            const qs_status st = pp.np[p] < 1 ? QS_E_INVAL : QS_E_UNSUPPORTED;
            return fail(st, "part %c has %d qubits (1 to %d)", p ? 'B' : 'A', pp.np[p], QS_MAX_QUBITS);
        }
    std::vector<qs::FlatOp> flat;
    std::string err;
    const int rc = qs::expand(c->ops, flat, err);
    if (rc == 2) return fail(QS_E_UNSUPPORTED, "%s", err.c_str());
    if (rc) return fail(QS_E_INVAL, "%s", err.c_str());
    auto local = [&](const std::vector<int> &qs_) {
        std::vector<int> r;
        for (int q : qs_) r.push_back(pp.pos[q]);
        return r;
    };
    for (auto &f : flat) {
        if (f.kind == qs::FlatOp::NOISE)
            return fail(QS_E_UNSUPPORTED, "noise sites in the partial-amplitude mode");
        int seen = 0;
        for (int q : f.targets) {
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
            seen |= 1 << pp.side[q];
        }
        for (int q : f.controls) {
            if (q >= n) return fail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
            seen |= 1 << pp.side[q];
        }
        if (seen != 3) {
            const int p = seen == 1 ? 0 : 1;
            pp.items.push_back({p, PartGate{local(f.targets), local(f.controls), f.m}});
            continue;
        }
        const qs::CanonGate g = qs::canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(),
                                                 int(f.controls.size()), f.m.data());
        if (g.kind == qs::CanonGate::IDENTITY) continue;
        PartCut cut;
        if (g.kind == qs::CanonGate::DENSE) {
            // targets in one part S; the controls in the other part become
            // the projector onto all ones (branch 1) or onto the rest
            const int S = pp.side[g.targets[0]];
            for (int q : g.targets)
                if (pp.side[q] != S)
                    return fail(QS_E_UNSUPPORTED, "a dense gate with targets on both sides of the dividing line");
            std::vector<int> cs, cp;
            for (int q : g.controls) (pp.side[q] == S ? cs : cp).push_back(q);
            if (cp.size() > QS_MAX_TARGETS)
                return fail(QS_E_UNSUPPORTED, "%zu controls across the dividing line", cp.size());
            const uint32_t ones = (1u << cp.size()) - 1;
            cut.pside = 1 - S;
            cut.proj[1] = diag_gate(local(cp), [&](uint32_t y) { return cd(y == ones ? 1.0 : 0.0); });
            cut.proj[0] = diag_gate(local(cp), [&](uint32_t y) { return cd(y == ones ? 0.0 : 1.0); });
            cut.other[1] = PartGate{local(g.targets), local(cs), g.m};
            cut.has[1] = true;
        } else {
            // a diagonal operator over Q = targets + controls: the factor of
            // the target pattern where every control is 1, else 1
            std::vector<int> Q = g.targets;
            Q.insert(Q.end(), g.controls.begin(), g.controls.end());
            int cnt[2] = {0, 0};
            for (int q : Q) cnt[pp.side[q]]++;
            const int ps = cnt[0] == 1 ? 0 : cnt[1] == 1 ? 1 : -1;
            if (ps < 0)
                return fail(QS_E_UNSUPPORTED, "a diagonal gate with more than one qubit on each side of the dividing line");
            if (cnt[1 - ps] > QS_MAX_TARGETS)
                return fail(QS_E_UNSUPPORTED, "a diagonal gate on more than %d qubits of one part", QS_MAX_TARGETS);
            int pq = -1;
            std::vector<int> rest;
            for (int q : Q) {
                if (pp.side[q] == ps)
                    pq = q;
                else
                    rest.push_back(q);
            }
            const int nt = int(g.targets.size());
            auto factor = [&](int pv, uint32_t y) {
                // value of qubit Q[i]: pv for the projector qubit, else its bit of y
                auto val = [&](int q) {
                    if (q == pq) return pv;
                    for (size_t i = 0; i < rest.size(); ++i)
                        if (rest[i] == q) return int((y >> (rest.size() - 1 - i)) & 1);
                    return 0;
                };
                for (int q : g.controls)
                    if (!val(q)) return cd(1.0);
                uint32_t x = 0;
                for (int b = 0; b < nt; ++b) x |= uint32_t(val(g.targets[b])) << (nt - 1 - b);
                return cd(g.m[2 * x], g.m[2 * x + 1]);
            };
            cut.pside = ps;
            for (int v = 0; v < 2; ++v) {
                cut.proj[v] = diag_gate({pp.pos[pq]}, [&](uint32_t y) { return cd(int(y) == v ? 1.0 : 0.0); });
                PartGate o = diag_gate(local(rest), [&](uint32_t y) { return factor(v, y); });
                bool ident = true;
                const size_t d = size_t(1) << rest.size();
                for (size_t y = 0; y < d; ++y)
                    ident = ident && o.m[2 * (y * d + y)] == 1.0 && o.m[2 * (y * d + y) + 1] == 0.0;
                cut.has[v] = !ident;
                if (!ident) cut.other[v] = std::move(o);
            }
        }
        pp.items.push_back({2 + int(pp.cuts.size()), PartGate{}});
        pp.cuts.push_back(std::move(cut));
    }
    if (pp.cuts.size() > QS_PARTIAL_MAX_CUTS)
        return fail(QS_E_UNSUPPORTED, "%zu gates cross the dividing line (at most %d)", pp.cuts.size(),
                    QS_PARTIAL_MAX_CUTS);
    return QS_OK;
}

// the sub-circuit of part p on branch word w
void partial_circuit(const PartialPlan &pp, int p, uint64_t w, qs_circuit &out)
{
    out.ops.clear();
    auto push = [&](const PartGate &g) {
        qs::Op op;
        op.kind = qs::Op::GATE;
        op.targets = g.t;
        op.controls = g.c;
        op.m = g.m;
        out.ops.push_back(std::move(op));
    };
    for (auto &it : pp.items) {
        if (it.first < 2) {
            if (it.first == p) push(it.second);
            continue;
        }
        const int j = it.first - 2;
        const PartCut &cut = pp.cuts[j];
        const int b = int((w >> j) & 1);
        if (cut.pside == p)
            push(cut.proj[b]);
        else if (cut.has[b])
            push(cut.other[b]);
    }
    out.changed();
}


// Device states of one run of the partial mode: `count` states of n qubits
// in buffers of their own, all enqueued on `strm`.
struct PartStates {
    std::vector<void *> bufs;
    std::vector<qs_state *> st;
    hipStream_t strm = nullptr;
    ~PartStates()
    {
        if (strm) hipStreamSynchronize(strm);  // nothing queued may still use them
        for (auto *s : st) qs_destroy(s);
        for (void *b : bufs) hipFree(b);
    }
    qs_status make(int n, qs_dtype dt, hipStream_t stream)
    {
        strm = stream;
        const size_t bytes = amp_bytes(dt) << n;
        void *b = nullptr;
        hipError_t e = hipMalloc(&b, bytes);
        if (e != hipSuccess)
            return e == hipErrorOutOfMemory ? fail(QS_E_NOMEM, "partial-amplitude state of %d qubits", n)
                                            : hip_fail(e, "hipMalloc");
        bufs.push_back(b);
        qs_state *s = nullptr;
        if (qs_status r = qs_create_from_buffer(n, dt, b, bytes, strm, &s)) return r;
        st.push_back(s);
        return QS_OK;
    }
};

qs_status apply_part_gate(qs_state *s, const PartGate &g)
{
    return qs_apply_gate(s, g.t.data(), int(g.t.size()), g.c.empty() ? nullptr : g.c.data(), int(g.c.size()),
                         g.m.data());
}

// Every branch word in turn: both sub-circuits from |0...0>, then one
// recombination term (memory: one state per part).
qs_status partial_branches(const PartialPlan &pp, qs_dtype dt, const qs_run_opts &o, const uint64_t *dix, size_t m,
                           double *acc, hipStream_t strm)
{
    PartStates ps;
    for (int p = 0; p < 2; ++p)
        if (qs_status r = ps.make(pp.np[p], dt, strm)) return r;
    qs_circuit sub[2];
    const uint64_t nw = uint64_t(1) << pp.cuts.size();
    for (uint64_t w = 0; w < nw; ++w) {
        for (int p = 0; p < 2; ++p) {
            partial_circuit(pp, p, w, sub[p]);
            if (qs_status r = qs_reset(ps.st[p])) return r;
            if (qs_status r = qs_run_circuit(ps.st[p], &sub[p], &o)) return r;
        }
        hipError_t e = qs::launch_partial_cmac(dt, ps.st[0]->amp, ps.st[1]->amp, dix, dix + m, m, acc, strm);
        if (e != hipSuccess) return hip_fail(e, "partial-amplitude recombination");
    }
    hipError_t e = hipStreamSynchronize(strm);
    return e == hipSuccess ? QS_OK : hip_fail(e, "partial-amplitude branches");
}

// Depth-first walk of the tree of cuts.  The gates of a part between cut
// j - 1 and cut j (segment j) do not depend on later branches, so the state
// after segment j is computed once per prefix of branch bits: a child starts
// from its parent's state (a copy for branch 0, the state itself for branch
// 1), receives cut j's operator for its branch and runs segment j + 1.  Each
// segment is one circuit whose plan is made once.  Memory: c + 1 states per
// part.
qs_status partial_tree(const PartialPlan &pp, qs_dtype dt, const qs_run_opts &o, const uint64_t *dix, size_t m,
                       double *acc, hipStream_t strm)
{
    const int c = int(pp.cuts.size());
    std::vector<std::unique_ptr<qs_circuit>> seg[2];
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k <= c; ++k) seg[p].emplace_back(new qs_circuit);
    int k = 0;
    for (auto &it : pp.items) {
        if (it.first >= 2) {
            k = it.first - 1;  // after cut j: segment j + 1
            continue;
        }
        qs::Op op;
        op.kind = qs::Op::GATE;
        op.targets = it.second.t;
        op.controls = it.second.c;
        op.m = it.second.m;
        seg[it.first][k]->ops.push_back(std::move(op));
    }
    PartStates ps[2];
    for (int p = 0; p < 2; ++p)
        for (int l = 0; l <= c; ++l)
            if (qs_status r = ps[p].make(pp.np[p], dt, strm)) return r;
    const size_t bytes[2] = {amp_bytes(dt) << pp.np[0], amp_bytes(dt) << pp.np[1]};
    for (int p = 0; p < 2; ++p)
        if (!seg[p][0]->ops.empty())
            if (qs_status r = qs_run_circuit(ps[p].st[0], seg[p][0].get(), &o)) return r;
    // walk(j, k): state slot k of each part holds the state after segment j
    // for the current prefix.  Branch 0 continues in a copy (slot k + 1);
    // branch 1 is the slot's last use, so it continues in place.  Slots stay
    // below c + 1: only branch-0 steps go one deeper.
    std::function<qs_status(int, int)> walk = [&](int j, int k) -> qs_status {
        if (j == c) {
            hipError_t e = qs::launch_partial_cmac(dt, ps[0].st[k]->amp, ps[1].st[k]->amp, dix, dix + m, m, acc, strm);
            return e == hipSuccess ? QS_OK : hip_fail(e, "partial-amplitude recombination");
        }
        const PartCut &cut = pp.cuts[j];
        for (int b = 0; b < 2; ++b) {
            const int kk = b == 0 ? k + 1 : k;
            for (int p = 0; p < 2; ++p) {
                qs_state *dst = ps[p].st[kk];
                if (kk != k) {
                    hipError_t e = hipMemcpyAsync(dst->amp, ps[p].st[k]->amp, bytes[p], hipMemcpyDeviceToDevice, strm);
                    if (e != hipSuccess) return hip_fail(e, "partial-amplitude state copy");
                }
                const PartGate *g = cut.pside == p ? &cut.proj[b] : cut.has[b] ? &cut.other[b] : nullptr;
                if (g)
                    if (qs_status r = apply_part_gate(dst, *g)) return r;
                if (!seg[p][j + 1]->ops.empty())
                    if (qs_status r = qs_run_circuit(dst, seg[p][j + 1].get(), &o)) return r;
            }
            if (qs_status r = walk(j + 1, kk)) return r;
        }
        return QS_OK;
    };
    qs_status r = walk(0, 0);
    hipError_t e = hipStreamSynchronize(strm);
    if (r) return r;
    return e == hipSuccess ? QS_OK : hip_fail(e, "partial-amplitude tree");
}

}  // namespace

qs_status qs_partial_cuts(const qs_circuit *c, int n, uint64_t part_a, int *cuts)
try {
    PartialPlan pp;
    if (qs_status st = build_partial(c, n, part_a, pp)) return st;
    if (cuts) *cuts = int(pp.cuts.size());
    return QS_OK;
} catch (const std::bad_alloc &) {
    return fail(QS_E_NOMEM, "host allocation failed while cutting the circuit");
}

qs_status qs_partial_amplitudes(const qs_circuit *c, int n, qs_dtype dt, uint64_t part_a, const uint64_t *idx,
                                size_t m, double *out, const qs_run_opts *opts, int *cuts)
try {
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", int(dt));
    if (m && (!idx || !out)) return fail(QS_E_INVAL, "idx or out is NULL");
    qs_run_opts o{};
    if (opts) o = *opts;
    if (o.plan == QS_PLAN_AUTOTUNE)
        return fail(QS_E_INVAL, "QS_PLAN_AUTOTUNE needs a circuit that runs repeatedly; every branch is a new one");
    if (o.plan < QS_PLAN_UNFUSED || o.plan > QS_PLAN_AUTOTUNE) return fail(QS_E_INVAL, "unknown plan %d", o.plan);
    PartialPlan pp;
    if (qs_status st = build_partial(c, n, part_a, pp)) return st;
    for (size_t k = 0; k < m; ++k)
        if (idx[k] >> n) return fail(QS_E_RANGE, "index %llu >= 2^%d", (unsigned long long)idx[k], n);
    if (cuts) *cuts = int(pp.cuts.size());
    if (m == 0) return QS_OK;
    // the bits of every index in part A and part B
    std::vector<uint64_t> ix[2];
    ix[0].resize(m);
    ix[1].resize(m);
    const size_t chunk = 1 << 14, nchunks = (m + chunk - 1) / chunk;
    parallel_for(nchunks, [&](size_t ci) {
        for (size_t k = ci * chunk; k < std::min(m, (ci + 1) * chunk); ++k) {
            uint64_t v[2] = {0, 0};
            for (int q = 0; q < n; ++q) v[pp.side[q]] |= ((idx[k] >> q) & 1) << pp.pos[q];
            ix[0][k] = v[0];
            ix[1][k] = v[1];
        }
    });
    // every state, copy and recombination runs in order on one stream
    hipStream_t strm = nullptr;
    uint64_t *dix = nullptr;
    double *acc = nullptr;
    auto cleanup = [&](qs_status r) {
        if (strm) hipStreamSynchronize(strm);
        if (dix) hipFree(dix);
        if (acc) hipFree(acc);
        if (strm) hipStreamDestroy(strm);
        return r;
    };
    hipError_t e = hipStreamCreateWithFlags(&strm, hipStreamNonBlocking);
    if (e != hipSuccess) {
        strm = nullptr;
        return hip_fail(e, "stream creation");
    }
    e = hipMalloc(&dix, 2 * m * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&acc, 2 * m * sizeof(double));
    if (e != hipSuccess)
        return cleanup(e == hipErrorOutOfMemory ? fail(QS_E_NOMEM, "partial-amplitude buffers for %zu indices", m)
                                                : hip_fail(e, "partial-amplitude set-up"));
    e = hipMemcpyAsync(dix, ix[0].data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, strm);
    if (e == hipSuccess) e = hipMemcpyAsync(dix + m, ix[1].data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, strm);
    if (e == hipSuccess) e = hipMemsetAsync(acc, 0, 2 * m * sizeof(double), strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    if (e != hipSuccess) return cleanup(hip_fail(e, "partial-amplitude set-up"));
    const size_t bytes[2] = {amp_bytes(dt) << pp.np[0], amp_bytes(dt) << pp.np[1]};
    const double tree_bytes = double(pp.cuts.size() + 1) * double(bytes[0] + bytes[1]);
    const size_t lim = g_mem_limit.load();
    const bool tree = tree_bytes <= kPartialTreeBytes && (lim == 0 || tree_bytes <= double(lim));
    qs_status r;
    try {
        r = tree ? partial_tree(pp, dt, o, dix, m, acc, strm) : partial_branches(pp, dt, o, dix, m, acc, strm);
    } catch (const std::bad_alloc &) {  // the buffers above are released before reporting
        r = fail(QS_E_NOMEM, "host allocation failed in the partial-amplitude mode");
    }
    if (r) return cleanup(r);
    e = hipMemcpyAsync(out, acc, 2 * m * sizeof(double), hipMemcpyDeviceToHost, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    if (e != hipSuccess) return cleanup(hip_fail(e, "partial-amplitude branches"));
    return cleanup(QS_OK);
} catch (const std::bad_alloc &) {
    return fail(QS_E_NOMEM, "host allocation failed in the partial-amplitude mode");
}

// -------------------------------------------------------------- readout --

qs_status qs_amplitudes(const qs_state *cs, const uint64_t *idx, size_t m, double *out)
try {
    qs_state *s = const_cast<qs_state *>(cs);
    if (qs_status st = check_state(s)) return st;
    if (!out && m) return fail(QS_E_INVAL, "out is NULL");
    const uint64_t na = uint64_t(1) << s->n;
    if (!idx) {
        if (m != na) return fail(QS_E_INVAL, "m = %zu but the state has %llu amplitudes", m, (unsigned long long)na);
        if (s->dt == QS_C128) {
            HIP_TRY(hipMemcpyAsync(out, s->amp, na * 16, hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
        } else {
            // the floats land in the upper half of `out` and are widened in
            // place from the front: double k (bytes 8k..8k+8) never reaches
            // an unread float (bytes from 8 na + 4 (k + 1)), so no staging
            // copy of the state is allocated
            unsigned char *base = reinterpret_cast<unsigned char *>(out);
            HIP_TRY(hipMemcpyAsync(base + 8 * na, s->amp, na * 8, hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
            for (uint64_t k = 0; k < 2 * na; ++k) {
                float f;
                std::memcpy(&f, base + 8 * na + 4 * k, 4);
                const double d = f;
                std::memcpy(base + 8 * k, &d, 8);
            }
        }
        return QS_OK;
    }
    for (size_t k = 0; k < m; ++k)
        if (idx[k] >= na) return fail(QS_E_RANGE, "index %llu >= 2^%d", (unsigned long long)idx[k], s->n);
    if (m == 0) return QS_OK;
    uint64_t *didx = nullptr;
    double *dvals = nullptr;
    HIP_TRY(hipMalloc(&didx, m * sizeof(uint64_t)));
    hipError_t e = hipMalloc(&dvals, m * 2 * sizeof(double));
    if (e != hipSuccess) {
        hipFree(didx);
        return hip_fail(e, "hipMalloc");
    }
    e = hipMemcpyAsync(didx, idx, m * sizeof(uint64_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = qs::launch_gather(s->dt, s->amp, didx, m, dvals, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dvals, m * 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    hipFree(didx);
    hipFree(dvals);
    if (e != hipSuccess) return hip_fail(e, "amplitude gather");
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_probabilities(const qs_state *cs, const int *qubits, int nq, double *out)
try {
    qs_state *s = const_cast<qs_state *>(cs);
    if (qs_status st = check_state(s)) return st;
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    std::vector<int> q;
    if (!qubits) {
        nq = s->n;
        for (int k = s->n - 1; k >= 0; --k) q.push_back(k);
    } else {
        if (qs_status st = check_qubits(s->n, qubits, nq, nullptr, 0, 30)) return st;
        q.assign(qubits, qubits + nq);
    }
    if (nq > 30) return fail(QS_E_UNSUPPORTED, "PMEASURE over more than 30 qubits");
    const size_t nb = size_t(1) << nq;
    double *dres = s->dout;
    const bool big = nb * sizeof(double) > 65536;
    if (big) HIP_TRY(hipMalloc(&dres, nb * sizeof(double)));
    hipError_t e;
    {
        Timed t(s, QS_K_REDUCE, double(amp_bytes(s->dt)) * std::ldexp(1.0, s->n), 3.0 * std::ldexp(1.0, s->n));
        e = qs::launch_probs(s->dt, s->amp, s->n, q.data(), nq, s->red, dres, s->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dres, nb * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (big) hipFree(dres);
    if (e != hipSuccess) return hip_fail(e, "probabilities");
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_probabilities_noalloc(const void *device_amps, int n, qs_dtype dt, const int *qubits, int nq,
                                   double *device_out, void *hip_stream)
{
    if (!device_amps || !device_out) return fail(QS_E_INVAL, "device_amps or device_out is NULL");
    if (n < 1 || n > QS_MAX_QUBITS) return fail(QS_E_INVAL, "n = %d not in [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", int(dt));
    if (reinterpret_cast<uintptr_t>(device_amps) % 16 || reinterpret_cast<uintptr_t>(device_out) % 8)
        return fail(QS_E_INVAL, "device_amps must be 16-byte and device_out 8-byte aligned");
    int q[QS_MAX_QUBITS];
    if (!qubits) {
        nq = n;
        for (int k = 0; k < n; ++k) q[k] = n - 1 - k;
    } else {
        if (qs_status st = check_qubits(n, qubits, nq, nullptr, 0, 30)) return st;
        for (int k = 0; k < nq; ++k) q[k] = qubits[k];
    }
    if (nq > 30) return fail(QS_E_UNSUPPORTED, "PMEASURE over more than 30 qubits");
    // the reductions that bin through the scratch take at most 1024 bins
    const size_t need = qs::reduce_scratch_doubles(n, nq <= 10 ? (1 << nq) : 1);
    if (need > qs::noalloc_scratch_doubles())
        return fail(QS_E_RANGE, "the reduction needs %zu scratch doubles, the static scratch holds %zu", need,
                    qs::noalloc_scratch_doubles());
    double *scr = nullptr;
    hipError_t e = qs::noalloc_scratch(&scr);
    if (e != hipSuccess) return hip_fail(e, "static reduction scratch");
    e = qs::launch_probs(dt, device_amps, n, q, nq, scr, device_out, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "probabilities");
    return QS_OK;
}

qs_status qs_norm(const qs_state *cs, double *out)
try {
    qs_state *s = const_cast<qs_state *>(cs);
    if (qs_status st = check_state(s)) return st;
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    {
        Timed t(s, QS_K_REDUCE, double(amp_bytes(s->dt)) * std::ldexp(1.0, s->n), 3.0 * std::ldexp(1.0, s->n));
        hipError_t e = qs::launch_norm2(s->dt, s->amp, s->n, s->red, s->dout, s->stream);
        if (e != hipSuccess) return hip_fail(e, "norm launch");
    }
    HIP_TRY(hipMemcpyAsync(s->hpin, s->dout, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    *out = s->hpin[0];
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_expect_z(const qs_state *cs, double *out)
try {
    qs_state *s = const_cast<qs_state *>(cs);
    if (qs_status st = check_state(s)) return st;
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    {
        Timed t(s, QS_K_REDUCE, double(amp_bytes(s->dt)) * std::ldexp(1.0, s->n),
                (3.0 + s->n) * std::ldexp(1.0, s->n));
        hipError_t e = qs::launch_expect_z(s->dt, s->amp, s->n, s->red, s->dout, s->stream);
        if (e != hipSuccess) return hip_fail(e, "expect_z launch");
    }
    HIP_TRY(hipMemcpyAsync(s->hpin, s->dout, s->n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::memcpy(out, s->hpin, s->n * sizeof(double));
    return QS_OK;
} QS_ABI_CATCH

// ---------------------------------------------------------- trajectories --

}  // extern "C"

namespace {

thread_local qs_traj_stats g_traj_stats{};

// Autotuning records of trajectory batches (QS_PLAN_AUTOTUNE), process-wide,
// keyed by dtype, batch size and the widths' range and total amplitudes.
struct TrajTuneKey {
    int dt, count, wmin, wmax;
    uint64_t amps;
    bool operator<(const TrajTuneKey &o) const
    {
        return std::tie(dt, count, wmin, wmax, amps) < std::tie(o.dt, o.count, o.wmin, o.wmax, o.amps);
    }
};
std::mutex g_traj_tune_mu;
std::map<TrajTuneKey, std::vector<double>> g_traj_tune;  // measured seconds per candidate (< 0: not yet run)

// Candidate widths of device-sampled passes: (qubits per tile, widest
// block, outer selector bits per op, trajectories per pass job); the first
// is the default.
const TrajParams kTrajCands[] = {{13, 4, 1, 128}, {13, 4, 1, 64}, {13, 4, 1, 0}, {13, 4, 2, 128},
                                 {13, 4, 2, 64},  {12, 4, 1, 128}, {13, 5, 1, 128}};
constexpr int kNumTrajCands = int(sizeof(kTrajCands) / sizeof(kTrajCands[0]));

}  // namespace

extern "C" {

qs_status qs_run_trajectories(const qs_circuit *const *circs, const int *widths, int count, qs_dtype dt,
                              uint64_t seed, const qs_run_opts *opts, double *z_out, double *traj_per_s)
try {
    g_traj_stats = qs_traj_stats{};
    qs_run_opts o{};
    if (opts) o = *opts;
    if (o.plan < QS_PLAN_UNFUSED || o.plan > QS_PLAN_AUTOTUNE) return fail(QS_E_INVAL, "unknown plan %d", o.plan);
    if (o.k_max && (o.k_max < 4 || o.k_max > 5))
        return fail(QS_E_INVAL, "k_max = %d: trajectory tiles take 4- or 5-qubit blocks (0 = default)", o.k_max);
    if (o.tile_qubits && (o.tile_qubits < 10 || o.tile_qubits > 13))
        return fail(QS_E_INVAL, "tile_qubits = %d not in [10, 13] (0 = default)", o.tile_qubits);
    if (!widths && count > 0) return fail(QS_E_INVAL, "widths is NULL");
    TrajParams par = kTrajCands[0];
    if (o.k_max) par.kmax = o.k_max;
    if (o.tile_qubits) par.m_cap = o.tile_qubits;
    int cand = -1;
    TrajTuneKey key{int(dt), count, 0, 0, 0};
    if (o.plan == QS_PLAN_AUTOTUNE && dt == QS_C64 && count > 0) {
        key.wmin = key.wmax = widths[0];
        for (int t = 0; t < count; ++t) {
            key.wmin = std::min(key.wmin, widths[t]);
            key.wmax = std::max(key.wmax, widths[t]);
            key.amps += (widths[t] >= 0 && widths[t] < 63) ? (uint64_t(1) << widths[t]) : 0;
        }
        std::lock_guard<std::mutex> lk(g_traj_tune_mu);
        auto &rec = g_traj_tune[key];
        if (rec.empty()) rec.assign(kNumTrajCands, -1.0);
        for (int c = 0; c < kNumTrajCands && cand < 0; ++c)
            if (rec[c] < 0) cand = c;
        if (cand < 0) {
            cand = 0;
            for (int c = 1; c < kNumTrajCands; ++c)
                if (rec[c] < rec[cand]) cand = c;
        }
        par = kTrajCands[cand];
    }
    qs_traj_stats st{};
    bool cold = false;
    const qs_status r = run_trajectory_batch(circs, widths, count, dt, seed, par, o.plan != QS_PLAN_UNFUSED,
                                             o.direct_launch == 0, z_out, st, cold);
    if (r) return r;
    if (cand >= 0) {
        std::lock_guard<std::mutex> lk(g_traj_tune_mu);
        auto &rec = g_traj_tune[key];
        // a call that enlarged the reused job buffers paid for allocations
        // later calls do not make: not recorded, the candidate runs again
        if (!cold && (rec[cand] < 0 || st.seconds < rec[cand])) rec[cand] = st.seconds;
        st.autotune_candidates = kNumTrajCands;
        for (double v : rec) st.autotune_tried += v >= 0;
    }
    g_traj_stats = st;
    if (traj_per_s) *traj_per_s = st.seconds > 0 ? double(count) / st.seconds : 0.0;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_trajectory_stats(qs_traj_stats *out)
{
    if (!out) return fail(QS_E_INVAL, "out is NULL");
    *out = g_traj_stats;
    return QS_OK;
}

// ------------------------------------------------------------ cost model --


qs_status qs_mlp_forward(const float *params, int f, int h, const float *x, int64_t n, float *y)
try {
    if (qs_status st = check_mlp(params, f, h)) return st;
    if (n < 0 || (n && (!x || !y))) return fail(QS_E_INVAL, "bad samples");
    if (n == 0) return QS_OK;
    const size_t np = qs::mlp_num_params(f, h);
    DevTmp t;
    float *dp, *dx, *dy;
    HIP_TRY(t.alloc(&dp, np));
    HIP_TRY(t.alloc(&dx, size_t(n) * f));
    HIP_TRY(t.alloc(&dy, size_t(n)));
    HIP_TRY(hipMemcpy(dp, params, np * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dx, x, size_t(n) * f * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(qs::launch_mlp_forward(dp, f, h, dx, n, dy, nullptr));
    HIP_TRY(hipMemcpy(y, dy, size_t(n) * sizeof(float), hipMemcpyDeviceToHost));
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_mlp_grad(const float *params, int f, int h, const float *x, const float *tv, int64_t n,
                      float *loss, float *grad)
try {
    if (qs_status st = check_mlp(params, f, h)) return st;
    if (n < 1 || !x || !tv || !loss || !grad) return fail(QS_E_INVAL, "bad samples");
    const size_t np = qs::mlp_num_params(f, h);
    DevTmp t;
    float *dp, *dx, *dt, *dg, *dl;
    HIP_TRY(t.alloc(&dp, np));
    HIP_TRY(t.alloc(&dx, size_t(n) * f));
    HIP_TRY(t.alloc(&dt, size_t(n)));
    HIP_TRY(t.alloc(&dg, np));
    HIP_TRY(t.alloc(&dl, 1));
    HIP_TRY(hipMemcpy(dp, params, np * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dx, x, size_t(n) * f * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dt, tv, size_t(n) * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(qs::launch_mlp_grad(dp, f, h, dx, dt, n, dg, dl, nullptr));
    HIP_TRY(hipMemcpy(grad, dg, np * sizeof(float), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(loss, dl, sizeof(float), hipMemcpyDeviceToHost));
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_mlp_train(float *params, int f, int h, const float *x, const float *tv, int64_t n, int steps,
                       int batch, float lr, uint64_t seed, float *loss)
try {
    if (qs_status st = check_mlp(params, f, h)) return st;
    if (n < 1 || !x || !tv) return fail(QS_E_INVAL, "bad samples");
    if (steps < 0 || batch < 1 || batch > 4096) return fail(QS_E_INVAL, "steps / batch out of range");
    if (!(lr > 0)) return fail(QS_E_INVAL, "learning rate must be positive");
    const size_t np = qs::mlp_num_params(f, h);
    // minibatch indices from the Philox stream (counter = draw index)
    std::vector<int> idx(size_t(steps) * batch);
    for (size_t i = 0; i < idx.size(); ++i)
        idx[i] = int(qs::noise_uniform(seed, 0xC057, i) * double(n)) % int(n);
    DevTmp t;
    float *dp, *dm, *dv, *dx, *dt, *dl;
    int *di;
    HIP_TRY(t.alloc(&dp, np));
    HIP_TRY(t.alloc(&dm, np));
    HIP_TRY(t.alloc(&dv, np));
    HIP_TRY(t.alloc(&dx, size_t(n) * f));
    HIP_TRY(t.alloc(&dt, size_t(n)));
    HIP_TRY(t.alloc(&dl, 1));
    HIP_TRY(t.alloc(&di, idx.size() + 1));
    HIP_TRY(hipMemcpy(dp, params, np * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(dm, 0, np * sizeof(float)));
    HIP_TRY(hipMemset(dv, 0, np * sizeof(float)));
    HIP_TRY(hipMemset(dl, 0, sizeof(float)));
    HIP_TRY(hipMemcpy(dx, x, size_t(n) * f * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dt, tv, size_t(n) * sizeof(float), hipMemcpyHostToDevice));
    if (!idx.empty()) HIP_TRY(hipMemcpy(di, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice));
    const int chunk = 256;  // steps per launch
    for (int s0 = 0; s0 < steps; s0 += chunk) {
        const int ns = std::min(chunk, steps - s0);
        HIP_TRY(qs::launch_mlp_train(dp, dm, dv, f, h, dx, dt, di + size_t(s0) * batch, batch, ns, s0, lr, dl,
                                     nullptr));
    }
    HIP_TRY(hipMemcpy(params, dp, np * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) HIP_TRY(hipMemcpy(loss, dl, sizeof(float), hipMemcpyDeviceToHost));
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_profile_samples(qs_state *s, float *features, float *y, int64_t capacity, int64_t *count)
try {
    if (qs_status st = check_state(s)) return st;
    if (capacity < 0 || (capacity && (!features || !y)) || !count) return fail(QS_E_INVAL, "bad output arrays");
    if (qs_status st = harvest(s)) return st;
    const int64_t c = std::min<int64_t>(capacity, int64_t(s->samples.size()));
    for (int64_t i = 0; i < c; ++i) {
        std::memcpy(features + i * QS_COST_FEATURES, s->samples[i].first.data(), sizeof(Features));
        y[i] = s->samples[i].second;
    }
    s->samples.erase(s->samples.begin(), s->samples.begin() + c);
    *count = c;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_cost_model_set(const float *params, int f, int h)
try {
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_model_version.fetch_add(1);
    if (!params) {
        g_model.clear();
        return QS_OK;
    }
    if (f != QS_COST_FEATURES) return fail(QS_E_INVAL, "the cost model takes %d features", QS_COST_FEATURES);
    if (h != qs::kMlpHidden) return fail(QS_E_UNSUPPORTED, "hidden width must be %d", qs::kMlpHidden);
    g_model.assign(params, params + qs::mlp_num_params(f, h));
    return QS_OK;
} QS_ABI_CATCH

// ------------------------------------------------------------- profiling --

qs_status qs_profile_enable(qs_state *s, int on)
try {
    if (qs_status st = check_state(s)) return st;
    s->prof = on != 0;
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_profile_reset(qs_state *s)
try {
    if (qs_status st = check_state(s)) return st;
    if (qs_status st = harvest(s)) return st;
    for (auto &a : s->acc) a = ProfAcc{};
    return QS_OK;
} QS_ABI_CATCH

qs_status qs_profile_query(qs_state *s, int kernel, int64_t *launches, double *total_ms,
                           double *alg_bytes, double *alg_flops)
try {
    if (qs_status st = check_state(s)) return st;
    if (kernel < 0 || kernel >= QS_K_COUNT) return fail(QS_E_INVAL, "unknown kernel class %d", kernel);
    if (qs_status st = harvest(s)) return st;
    const ProfAcc &a = s->acc[kernel];
    if (launches) *launches = a.launches;
    if (total_ms) *total_ms = a.ms;
    if (alg_bytes) *alg_bytes = a.bytes;
    if (alg_flops) *alg_flops = a.flops;
    return QS_OK;
} QS_ABI_CATCH

}  // extern "C"

namespace qs {
qs_status set_error(qs_status st, const char *msg) { return fail(st, "%s", msg); }
const std::vector<Op> &circuit_ops(const qs_circuit *c) { return c->ops; }
std::shared_ptr<const void> circuit_cache_get(const qs_circuit *c, uint64_t key)
{
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->other.find(key);
    return it == c->other.end() ? nullptr : it->second;
}
void circuit_cache_put(const qs_circuit *c, uint64_t key, std::shared_ptr<const void> v)
{
    std::lock_guard<std::mutex> lk(c->mu);
    c->other[key] = std::move(v);
}
size_t memory_limit() { return g_mem_limit.load(); }
qs_status run_on_state(qs_state *s, const qs_circuit *c, const qs_run_opts *o) { return qs_run_circuit(s, c, o); }
}  // namespace qs
