// Group expansion, gate canonicalisation, greedy fusion and the trajectory
// runner (host side of libqs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "qs_philox.h"
#include "qs_plan.h"

using cd = std::complex<double>;

namespace qs {

namespace {

int find_group_end(const std::vector<Op> &ops, size_t open, size_t hi)
{
    int depth = 0;
    for (size_t k = open; k < hi; ++k) {
        const Op::Kind kd = ops[k].kind;
        if (kd == Op::BEGIN_DAGGER || kd == Op::BEGIN_CONTROL) ++depth;
        if (kd == Op::END_DAGGER || kd == Op::END_CONTROL) {
            if (--depth == 0) return int(k);
        }
    }
    return -1;
}

int expand_range(const std::vector<Op> &ops, size_t lo, size_t hi, bool in_group,
                 std::vector<FlatOp> &out, std::string &err)
{
    for (size_t k = lo; k < hi; ++k) {
        const Op &op = ops[k];
        if (op.kind == Op::GATE) {
            FlatOp f;
            f.kind = FlatOp::GATE;
            f.targets = op.targets;
            f.controls = op.controls;
            f.m = op.m;
            out.push_back(std::move(f));
        } else if (op.kind == Op::NOISE) {
            if (in_group) {
                err = "noise site inside a DAGGER or CONTROL group";
                return 2;
            }
            FlatOp f;
            f.kind = FlatOp::NOISE;
            f.targets = op.targets;
            f.m = op.m;
            f.nk = op.nk;
            out.push_back(std::move(f));
        } else if (op.kind == Op::BEGIN_DAGGER || op.kind == Op::BEGIN_CONTROL) {
            const int e = find_group_end(ops, k, hi);
            if (e < 0) {
                err = "unbalanced DAGGER / CONTROL group";
                return 1;
            }
            const bool dag = op.kind == Op::BEGIN_DAGGER;
            if (dag != (ops[e].kind == Op::END_DAGGER)) {
                err = "DAGGER and CONTROL groups are interleaved";
                return 1;
            }
            std::vector<FlatOp> inner;
            if (int rc = expand_range(ops, k + 1, size_t(e), true, inner, err)) return rc;
            if (dag) {
                // the inverse of G_1 ... G_m is G_m^dagger ... G_1^dagger
                for (auto it = inner.rbegin(); it != inner.rend(); ++it) {
                    FlatOp g = *it;
                    const int d = 1 << g.targets.size();
                    std::vector<double> mt(g.m.size());
                    for (int r = 0; r < d; ++r)
                        for (int c = 0; c < d; ++c) {
                            mt[2 * (r * d + c)] = g.m[2 * (c * d + r)];
                            mt[2 * (r * d + c) + 1] = -g.m[2 * (c * d + r) + 1];
                        }
                    g.m = std::move(mt);
                    out.push_back(std::move(g));
                }
            } else {
                for (auto &g : inner) {
                    for (int q : g.targets)
                        if (q == op.qubit) {
                            err = "CONTROL qubit is also a target inside its group";
                            return 1;
                        }
                    for (int q : g.controls)
                        if (q == op.qubit) {
                            err = "CONTROL qubit is repeated inside its group";
                            return 1;
                        }
                    g.controls.push_back(op.qubit);
                    out.push_back(std::move(g));
                }
            }
            k = size_t(e);
        } else {
            err = "ENDDAGGER / ENDCONTROL without an opening marker";
            return 1;
        }
    }
    return 0;
}

inline cd at(const std::vector<cd> &M, int d, int r, int c) { return M[size_t(r) * d + c]; }

// Apply a gate given on local bits to every column of the block matrix.
// Local bit L of a block index corresponds to block qubit position L.
void apply_local(std::vector<cd> &M, int k, const std::vector<int> &tbits,
                 const std::vector<int> &cbits, const std::vector<double> &m)
{
    const int D = 1 << k;
    const int nt = int(tbits.size());
    const int g = 1 << nt;
    int tmask = 0, cmask = 0;
    for (int b : tbits) tmask |= 1 << b;
    for (int b : cbits) cmask |= 1 << b;
    std::vector<int> off(g);
    for (int x = 0; x < g; ++x) {
        int o = 0;
        for (int b = 0; b < nt; ++b)
            if ((x >> (nt - 1 - b)) & 1) o |= 1 << tbits[b];
        off[x] = o;
    }
    std::vector<cd> v(g), w(g);
    for (int col = 0; col < D; ++col)
        for (int i = 0; i < D; ++i) {
            if ((i & tmask) || (i & cmask) != cmask) continue;
            for (int x = 0; x < g; ++x) v[x] = M[size_t(i | off[x]) * D + col];
            for (int r = 0; r < g; ++r) {
                cd acc = 0;
                for (int c = 0; c < g; ++c) acc += cd(m[2 * (r * g + c)], m[2 * (r * g + c) + 1]) * v[c];
                w[r] = acc;
            }
            for (int x = 0; x < g; ++x) M[size_t(i | off[x]) * D + col] = w[x];
        }
}

struct Block {
    uint64_t qmask = 0;
    std::vector<size_t> gates;  // indices into flat
    size_t first = 0;           // creation order
};

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace

int expand(const std::vector<Op> &ops, std::vector<FlatOp> &out, std::string &err)
{
    out.clear();
    return expand_range(ops, 0, ops.size(), false, out, err);
}

bool is_identity(const std::vector<double> &m, int nt)
{
    const int d = 1 << nt;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const double re = m[2 * (r * d + c)], im = m[2 * (r * d + c) + 1];
            if (re != (r == c ? 1.0 : 0.0) || im != 0.0) return false;
        }
    return true;
}

CanonGate canonicalize(const int *t, int nt, const int *c, int nc, const double *m)
{
    std::vector<int> tg(t, t + nt), ct(c, c + nc);
    int d = 1 << nt;
    std::vector<cd> M(size_t(d) * d);
    for (int k = 0; k < d * d; ++k) M[k] = cd(m[2 * k], m[2 * k + 1]);
    // Pull out targets that act as |1>-controls (Eq. 3 form).
    bool changed = true;
    while (changed && !tg.empty()) {
        changed = false;
        const int cur = int(tg.size());
        for (int b = 0; b < cur; ++b) {
            const int sh = cur - 1 - b;
            bool ctl = true;
            for (int r = 0; r < d && ctl; ++r)
                for (int cc = 0; cc < d && ctl; ++cc) {
                    if (((r >> sh) & 1) && ((cc >> sh) & 1)) continue;
                    const cd want = (r == cc) ? cd(1) : cd(0);
                    if (at(M, d, r, cc) != want) ctl = false;
                }
            if (!ctl) continue;
            const int nd = d / 2;
            std::vector<cd> R(size_t(nd) * nd);
            auto squeeze = [&](int x) {  // index with bit sh removed
                const int lo = x & ((1 << sh) - 1);
                return ((x >> (sh + 1)) << sh) | lo;
            };
            for (int r = 0; r < d; ++r)
                for (int cc = 0; cc < d; ++cc)
                    if (((r >> sh) & 1) && ((cc >> sh) & 1)) R[size_t(squeeze(r)) * nd + squeeze(cc)] = at(M, d, r, cc);
            ct.push_back(tg[b]);
            tg.erase(tg.begin() + b);
            M.swap(R);
            d = nd;
            changed = true;
            break;
        }
    }
    CanonGate g;
    g.targets = tg;
    g.controls = ct;
    const int n2 = int(tg.size());
    bool diag = true, ident = true;
    for (int r = 0; r < d; ++r)
        for (int cc = 0; cc < d; ++cc) {
            const cd v = at(M, d, r, cc);
            if (r != cc && v != cd(0)) diag = false;
            if (v != ((r == cc) ? cd(1) : cd(0))) ident = false;
        }
    if (ident) {
        g.kind = CanonGate::IDENTITY;
        return g;
    }
    if (diag) {
        g.kind = CanonGate::PHASE;
        g.m.resize(size_t(2) * d);
        for (int x = 0; x < d; ++x) {
            g.m[2 * x] = at(M, d, x, x).real();
            g.m[2 * x + 1] = at(M, d, x, x).imag();
        }
        return g;
    }
    (void)n2;
    g.kind = CanonGate::DENSE;
    g.m.resize(size_t(2) * d * d);
    for (int k = 0; k < d * d; ++k) {
        g.m[2 * k] = M[k].real();
        g.m[2 * k + 1] = M[k].imag();
    }
    return g;
}

int default_kmax(int n, qs_dtype dt)
{
    (void)n;
    (void)dt;
    return 4;
}

// Greedy fusion over the gate sequence: open blocks own disjoint qubit sets;
// a gate joins (and merges) the blocks owning its qubits when the union fits
// in kmax qubits, otherwise those blocks are closed (emitted) and the gate
// opens a new block.  Blocks on disjoint qubits commute, so emitting a block
// when it closes keeps every gate after the gates it depends on.
void greedy_fuse(const std::vector<FlatOp> &flat, size_t k0, size_t e, int kmax,
                 std::vector<CanonGate> &plan)
{
    std::vector<std::unique_ptr<Block>> open;
    auto emit = [&](Block &b) {
        if (b.gates.size() == 1) {
            const FlatOp &f = flat[b.gates[0]];
            plan.push_back(canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(),
                                        int(f.controls.size()), f.m.data()));
            return;
        }
        std::vector<int> qs;
        for (int q = 63; q >= 0; --q)
            if (b.qmask >> q & 1) qs.push_back(q);  // qs[0] = highest qubit = MSB
        const int k = int(qs.size());
        const int D = 1 << k;
        auto local = [&](int q) {
            for (int i = 0; i < k; ++i)
                if (qs[i] == q) return k - 1 - i;
            return -1;
        };
        std::vector<cd> M(size_t(D) * D, cd(0));
        for (int i = 0; i < D; ++i) M[size_t(i) * D + i] = 1;
        for (size_t gi : b.gates) {
            const FlatOp &f = flat[gi];
            std::vector<int> tb, cb;
            for (int q : f.targets) tb.push_back(local(q));
            for (int q : f.controls) cb.push_back(local(q));
            apply_local(M, k, tb, cb, f.m);
        }
        std::vector<double> mm(size_t(2) * D * D);
        for (int i = 0; i < D * D; ++i) {
            mm[2 * i] = M[i].real();
            mm[2 * i + 1] = M[i].imag();
        }
        plan.push_back(canonicalize(qs.data(), k, nullptr, 0, mm.data()));
    };
    size_t serial = 0;
    for (size_t gi = k0; gi < e; ++gi) {
        const FlatOp &f = flat[gi];
        uint64_t q = 0;
        for (int t : f.targets) q |= uint64_t(1) << t;
        for (int c : f.controls) q |= uint64_t(1) << c;
        std::vector<size_t> hit;
        uint64_t uni = q;
        for (size_t b = 0; b < open.size(); ++b)
            if (open[b]->qmask & q) {
                hit.push_back(b);
                uni |= open[b]->qmask;
            }
        if (popcount64(uni) <= kmax) {
            auto nb = std::make_unique<Block>();
            nb->qmask = uni;
            nb->first = serial++;
            // merge in the order the blocks were opened
            std::sort(hit.begin(), hit.end(), [&](size_t a, size_t b) { return open[a]->first < open[b]->first; });
            for (size_t b : hit)
                nb->gates.insert(nb->gates.end(), open[b]->gates.begin(), open[b]->gates.end());
            nb->gates.push_back(gi);
            if (!hit.empty()) nb->first = open[hit[0]]->first;
            std::vector<std::unique_ptr<Block>> keep;
            for (size_t b = 0; b < open.size(); ++b)
                if (std::find(hit.begin(), hit.end(), b) == hit.end()) keep.push_back(std::move(open[b]));
            keep.push_back(std::move(nb));
            open.swap(keep);
            continue;
        }
        // close the blocks that share qubits with this gate
        std::sort(hit.begin(), hit.end(), [&](size_t a, size_t b) { return open[a]->first < open[b]->first; });
        for (size_t b : hit) emit(*open[b]);
        std::vector<std::unique_ptr<Block>> keep;
        for (size_t b = 0; b < open.size(); ++b)
            if (std::find(hit.begin(), hit.end(), b) == hit.end()) keep.push_back(std::move(open[b]));
        open.swap(keep);
        if (popcount64(q) > kmax) {
            plan.push_back(canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(),
                                        int(f.controls.size()), f.m.data()));
        } else {
            auto nb = std::make_unique<Block>();
            nb->qmask = q;
            nb->first = serial++;
            nb->gates.push_back(gi);
            open.push_back(std::move(nb));
        }
    }
    std::sort(open.begin(), open.end(), [](const std::unique_ptr<Block> &a, const std::unique_ptr<Block> &b) {
        return a->first < b->first;
    });
    for (auto &b : open) emit(*b);
}

// Sequential trajectory runner: one state per distinct width, reused.
qs_status run_trajectories(const qs_circuit *const *circs, const int *widths, int count, qs_dtype dt,
                           uint64_t seed, double *z_out, double *seconds)
{
    if (!circs || !widths || !z_out || count < 0) return set_error(QS_E_INVAL, "NULL argument or negative count");
    std::map<int, qs_state *> states;
    auto cleanup = [&]() {
        for (auto &kv : states) qs_destroy(kv.second);
    };
    const auto t0 = std::chrono::steady_clock::now();
    size_t off = 0;
    for (int t = 0; t < count; ++t) {
        const int n = widths[t];
        if (n < 1 || n > QS_MAX_QUBITS) {
            cleanup();
            return set_error(QS_E_INVAL, "trajectory width out of range");
        }
        qs_state *s = nullptr;
        auto it = states.find(n);
        if (it == states.end()) {
            if (qs_status st = qs_create(n, dt, &s)) {
                cleanup();
                return st;
            }
            states[n] = s;
        } else {
            s = it->second;
            if (qs_status st = qs_reset(s)) {
                cleanup();
                return st;
            }
        }
        qs_run_opts o{};
        o.plan = QS_PLAN_UNFUSED;
        o.seed = seed;
        o.traj = uint64_t(t);
        if (qs_status st = run_on_state(s, circs[t], &o)) {
            cleanup();
            return st;
        }
        if (qs_status st = qs_expect_z(s, z_out + off)) {
            cleanup();
            return st;
        }
        off += size_t(n);
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (seconds) *seconds = std::chrono::duration<double>(t1 - t0).count();
    cleanup();
    return QS_OK;
}

}  // namespace qs

extern "C" {

double qs_philox_uniform(uint64_t seed, uint64_t traj, uint64_t site)
{
    return qs::noise_uniform(seed, traj, site);
}

void qs_philox4x32_10(const uint32_t *counter, const uint32_t *key, uint32_t *out)
{
    if (!counter || !key || !out) return;
    qs::Philox4 c;
    for (int k = 0; k < 4; ++k) c.w[k] = counter[k];
    const qs::Philox4 r = qs::philox4x32_10(c, key[0], key[1]);
    for (int k = 0; k < 4; ++k) out[k] = r.w[k];
}

}  // extern "C"
