// Single-amplitude mode (Sec. 2.3, Figs. 2-3): host side.
//
// The circuit becomes an undirected graphical model.  Every Boolean
// variable (the value of one qubit between two gates that may change it) is
// a vertex; every non-identity gate is one edge, a tensor over the vertices
// it touches:
//  - a diagonal gate (after pulling |1>-controls out of the matrix) keeps the
//    variables of its qubits: a tensor over their current vertices whose
//    entries are the diagonal factors (1 where a control reads 0);
//  - any other gate gives each target a new vertex: a tensor over (new
//    target vertices, old target vertices, control vertices) with entries
//    U[new, old] where every control reads 1 and delta(new, old) elsewhere
//    (the row index of U is the value after the gate).
// The first vertex of every qubit is fixed to 0 (the initial state) and its
// last to the measured bit (differential elimination without doubling);
// the nslice free vertices on the most edges are fixed as well, giving 2^nslice
// graphs that run side by side as a batch and are summed at the end.  Every
// other vertex is eliminated: the tensors on it are merged pairwise in order
// of rank and the vertex is summed out with the last merge (integral
// elimination), together with any other vertex that no further tensor holds.
// Which vertex goes next is chosen greedily, the one whose merged tensor is
// smallest.  What remains are scalars; their product per graph, summed over
// the graphs, is the amplitude.  The merges run on the device (qs_single.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "qs_internal.h"
#include "qs_plan.h"
#include "qs_single.h"

using cd = std::complex<double>;

namespace {

qs_status sfail(qs_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return qs::set_error(st, buf);
}

enum VKind { V_FREE = 0, V_INPUT = 1, V_OUTPUT = 2, V_SLICE = 3 };

struct Vert {
    int qubit = -1;
    int kind = V_FREE;
    int which = 0;  // V_OUTPUT: the qubit (bit of the bitstring); V_SLICE: bit of the slice number
};

// A gate's tensor as built on the host: bit j of the index is vertex idx[j].
struct Base {
    std::vector<int> idx;
    std::vector<cd> v;
};

struct Ten {
    std::vector<int> idx;     // free vertices (a set)
    bool batched = false;     // depends on the bitstring or the slice
    int base = -1;            // initial tensor: its Base; -1 = made by a merge
    std::vector<int> layout;  // storage order asked for by its consumer, lowest bit first
    bool own_low = false;     // as an operand: its own vertices lowest, then the summed ones
    int producer = -1;        // the merge that makes it (-1 = initial tensor)
};

struct Merge {
    int x, y, z;
    std::vector<int> b, m, n, k;  // shared kept, x only, y only (each in the order of z's storage), summed
};

struct Plan {
    int n = 0;
    std::vector<Vert> verts;
    std::vector<Base> bases;
    std::vector<Ten> tens;
    std::vector<Merge> merges;
    std::vector<int> finals;  // tensors left as scalars
    uint64_t idle = 0;        // qubits whose first vertex is also their last
    int nslice = 0;
    int fixed = 0;
    int max_rank = 0;
    double flops1 = 0;        // real flops of the merges for one batch element (batched merges) ...
    double flops0 = 0;        // ... and once per call (unbatched merges)
};

// ------------------------------------------------------------ the graph --

qs_status build_graph(const qs_circuit *c, int n, int nslice, Plan &P)
{
    if (n < 1 || n > QS_MAX_CIRCUIT_QUBITS) return sfail(QS_E_INVAL, "n = %d not in [1, %d]", n, QS_MAX_CIRCUIT_QUBITS);
    if (nslice < 0 || nslice > QS_SINGLE_MAX_SLICES)
        return sfail(QS_E_INVAL, "nslice = %d not in [0, %d]", nslice, QS_SINGLE_MAX_SLICES);
    std::vector<qs::FlatOp> flat;
    std::string err;
    const int rc = qs::expand(qs::circuit_ops(c), flat, err);
    if (rc) return sfail(rc == 2 ? QS_E_UNSUPPORTED : QS_E_INVAL, "%s", err.c_str());
    P.n = n;
    std::vector<int> cur(n);
    for (int q = 0; q < n; ++q) {
        Vert v;
        v.qubit = q;
        v.kind = V_INPUT;
        cur[q] = int(P.verts.size());
        P.verts.push_back(v);
    }
    std::vector<int> first = cur;
    for (const auto &f : flat) {
        if (f.kind == qs::FlatOp::NOISE)
            return sfail(QS_E_UNSUPPORTED, "the single-amplitude mode takes unitary circuits (noise site found)");
        for (int q : f.targets)
            if (q >= n) return sfail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        for (int q : f.controls)
            if (q >= n) return sfail(QS_E_RANGE, "qubit %d out of range [0, %d)", q, n);
        const qs::CanonGate g = qs::canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(),
                                                 int(f.controls.size()), f.m.data());
        if (g.kind == qs::CanonGate::IDENTITY) continue;
        const int nt = int(g.targets.size()), nc = int(g.controls.size());
        Base B;
        if (g.kind == qs::CanonGate::PHASE) {
            // Fig. 2 (a), (c): the vertices of the qubits are kept
            for (int t : g.targets) B.idx.push_back(cur[t]);
            for (int q : g.controls) B.idx.push_back(cur[q]);
            const int r = nt + nc;
            B.v.assign(size_t(1) << r, cd(1.0, 0.0));
            for (uint32_t i = 0; i < (1u << r); ++i) {
                bool on = true;
                for (int j = 0; j < nc; ++j) on = on && ((i >> (nt + j)) & 1u);
                if (!on) continue;
                uint32_t x = 0;  // diagonal index: targets[0] is the most significant bit
                for (int b = 0; b < nt; ++b) x |= ((i >> b) & 1u) << (nt - 1 - b);
                B.v[i] = cd(g.m[2 * x], g.m[2 * x + 1]);
            }
        } else {
            // Fig. 2 (b), (d): a new vertex for every target
            std::vector<int> nv(nt);
            for (int b = 0; b < nt; ++b) {
                Vert v;
                v.qubit = g.targets[b];
                nv[b] = int(P.verts.size());
                P.verts.push_back(v);
            }
            for (int b = 0; b < nt; ++b) B.idx.push_back(nv[b]);
            for (int t : g.targets) B.idx.push_back(cur[t]);
            for (int q : g.controls) B.idx.push_back(cur[q]);
            const int r = 2 * nt + nc, d = 1 << nt;
            if (r > 24) return sfail(QS_E_UNSUPPORTED, "gate with %d targets and %d controls", nt, nc);
            B.v.assign(size_t(1) << r, cd(0.0, 0.0));
            for (uint32_t i = 0; i < (1u << r); ++i) {
                bool on = true;
                for (int j = 0; j < nc; ++j) on = on && ((i >> (2 * nt + j)) & 1u);
                uint32_t row = 0, col = 0;
                for (int b = 0; b < nt; ++b) {
                    row |= ((i >> b) & 1u) << (nt - 1 - b);
                    col |= ((i >> (nt + b)) & 1u) << (nt - 1 - b);
                }
                if (on)
                    B.v[i] = cd(g.m[2 * (size_t(row) * d + col)], g.m[2 * (size_t(row) * d + col) + 1]);
                else
                    B.v[i] = row == col ? cd(1.0, 0.0) : cd(0.0, 0.0);
            }
            for (int b = 0; b < nt; ++b) cur[g.targets[b]] = nv[b];
        }
        P.bases.push_back(std::move(B));
    }
    // the measured bit fixes each qubit's last vertex
    for (int q = 0; q < n; ++q) {
        if (cur[q] == first[q]) {
            P.idle |= uint64_t(1) << q;  // fixed to 0 as the initial vertex; bit q must be 0
            continue;
        }
        P.verts[cur[q]].kind = V_OUTPUT;
        P.verts[cur[q]].which = q;
    }
    // slicing: the free vertices on the most edges (Sec. 2.3, third step)
    std::vector<int> deg(P.verts.size(), 0);
    for (const auto &B : P.bases)
        for (int v : B.idx) ++deg[v];
    std::vector<int> cand;
    for (size_t v = 0; v < P.verts.size(); ++v)
        if (P.verts[v].kind == V_FREE) cand.push_back(int(v));
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return deg[a] > deg[b]; });
    P.nslice = std::min<int>(nslice, int(cand.size()));
    for (int i = 0; i < P.nslice; ++i) {
        P.verts[cand[i]].kind = V_SLICE;
        P.verts[cand[i]].which = i;
    }
    for (const auto &v : P.verts) P.fixed += v.kind != V_FREE;
    return QS_OK;
}

// ------------------------------------------------------- elimination order --

// Tie-break between vertices of equal merged size: a hash of (vertex,
// trial), so that each trial of the greedy order explores another order.
uint64_t tie_key(int v, int trial)
{
    uint64_t x = (uint64_t(uint32_t(v)) << 32) ^ uint64_t(uint32_t(trial)) * 0x9E3779B97F4A7C15ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    return trial == 0 ? uint64_t(v) : x;
}

qs_status plan_merges(Plan &P, int trial)
{
    const int nv = int(P.verts.size());
    std::vector<std::set<int>> on(nv);  // alive tensors holding each free vertex
    auto add_tensor = [&](Ten t) {
        const int id = int(P.tens.size());
        for (int v : t.idx) on[v].insert(id);
        P.tens.push_back(std::move(t));
        return id;
    };
    for (size_t bi = 0; bi < P.bases.size(); ++bi) {
        Ten t;
        t.base = int(bi);
        for (int v : P.bases[bi].idx) {
            const int k = P.verts[v].kind;
            if (k == V_FREE) t.idx.push_back(v);
            if (k == V_OUTPUT || k == V_SLICE) t.batched = true;
        }
        std::sort(t.idx.begin(), t.idx.end());
        add_tensor(std::move(t));
    }
    std::vector<char> alive(P.tens.size(), 1);
    std::set<int> left;
    for (int v = 0; v < nv; ++v)
        if (P.verts[v].kind == V_FREE) left.insert(v);
    const double bt_est = std::ldexp(1.0, P.nslice);
    auto merged_cost = [&](int v, int &rank) {
        std::set<int> u;
        bool batched = false;
        for (int t : on[v]) {
            u.insert(P.tens[t].idx.begin(), P.tens[t].idx.end());
            batched = batched || P.tens[t].batched;
        }
        rank = int(u.size()) - 1;
        return std::ldexp(batched ? bt_est : 1.0, rank);
    };
    while (!left.empty()) {
        int best = -1, best_rank = 0;
        double best_cost = 0;
        for (int v : left) {
            int r;
            const double cst = merged_cost(v, r);
            if (best < 0 || cst < best_cost ||
                (cst == best_cost && (on[v].size() < on[best].size() ||
                                      (on[v].size() == on[best].size() && tie_key(v, trial) < tie_key(best, trial))))) {
                best = v;
                best_cost = cst;
                best_rank = r;
            }
        }
        if (best_rank > qs::kSaMaxBits - 6)
            return sfail(QS_E_NOMEM, "the elimination needs a tensor of %d indices", best_rank);
        std::vector<int> group(on[best].begin(), on[best].end());
        if (group.size() == 1) {
            // a vertex on one edge only: summed against a vector of ones
            const int bi = int(P.bases.size());
            Base ones;
            ones.idx = {best};
            ones.v = {cd(1.0, 0.0), cd(1.0, 0.0)};
            P.bases.push_back(ones);
            Ten t;
            t.base = bi;
            t.idx = {best};
            group.push_back(add_tensor(std::move(t)));
            alive.push_back(1);
        }
        std::stable_sort(group.begin(), group.end(),
                         [&](int a, int b) { return P.tens[a].idx.size() < P.tens[b].idx.size(); });
        int acc = group[0];
        for (size_t i = 1; i < group.size(); ++i) {
            const int x = acc, y = group[i];
            const Ten &X = P.tens[x], &Y = P.tens[y];
            Merge M;
            M.x = x;
            M.y = y;
            std::set<int> ys(Y.idx.begin(), Y.idx.end()), xs(X.idx.begin(), X.idx.end());
            for (int v : X.idx) {
                if (!ys.count(v)) {
                    M.m.push_back(v);
                    continue;
                }
                // summed when no other alive tensor holds it
                bool other = false;
                for (int t : on[v])
                    if (t != x && t != y) other = true;
                (other ? M.b : M.k).push_back(v);
            }
            for (int v : Y.idx)
                if (!xs.count(v)) M.n.push_back(v);
            Ten z;
            z.batched = X.batched || Y.batched;
            z.idx = M.b;
            z.idx.insert(z.idx.end(), M.m.begin(), M.m.end());
            z.idx.insert(z.idx.end(), M.n.begin(), M.n.end());
            std::sort(z.idx.begin(), z.idx.end());
            const double outs = std::ldexp(1.0, int(M.b.size() + M.m.size() + M.n.size()));
            const double f = 8.0 * outs * std::ldexp(1.0, int(M.k.size()));
            (z.batched ? P.flops1 : P.flops0) += f;
            P.max_rank = std::max(P.max_rank, int(z.idx.size()));
            for (int v : X.idx) on[v].erase(x);
            for (int v : Y.idx) on[v].erase(y);
            alive[x] = alive[y] = 0;
            for (int v : M.k) left.erase(v);
            z.producer = int(P.merges.size());
            M.z = add_tensor(std::move(z));
            alive.push_back(1);
            P.merges.push_back(std::move(M));
            acc = P.merges.back().z;
        }
    }
    for (size_t t = 0; t < P.tens.size(); ++t)
        if (alive[t]) {
            if (!P.tens[t].idx.empty()) return sfail(QS_E_DEVICE, "internal: tensor %zu left with indices", t);
            P.finals.push_back(int(t));
        }
    // Storage order of every operand, as its merge reads it: the summed
    // vertices and the operand's own vertices in the low bits (either group
    // lowest), then the shared kept ones.  A merge writes its result in the
    // order its consumer reads it, so the merges are walked from the last:
    // each one's vertex lists are ordered by their places in its result's
    // storage (the consumer, later in the list, has fixed it) and the operand
    // whose own vertices hold the lowest storage bit takes the fastest index
    // n, so that neighbouring threads write neighbouring addresses.  For an
    // operand made by an earlier merge, the group put lowest is the one
    // whose leading vertices that merge writes from its tiled (own) index
    // ranges rather than its batch of shared vertices.
    for (size_t i = P.merges.size(); i-- > 0;) {
        Merge &M = P.merges[i];
        const Ten &Z = P.tens[M.z];
        if (!Z.layout.empty()) {
            std::map<int, int> pos;
            for (size_t j = 0; j < Z.layout.size(); ++j) pos[Z.layout[j]] = int(j);
            auto by_pos = [&](std::vector<int> &v) {
                std::sort(v.begin(), v.end(), [&](int a, int b) { return pos[a] < pos[b]; });
            };
            by_pos(M.b);
            by_pos(M.m);
            by_pos(M.n);
            const int v0 = Z.layout[0];
            if (std::find(M.m.begin(), M.m.end(), v0) != M.m.end()) {
                std::swap(M.x, M.y);
                std::swap(M.m, M.n);
            }
        }
        auto lay = [&](Ten &T, const std::vector<int> &own) {
            std::vector<int> klow = M.k, olow = own;
            klow.insert(klow.end(), own.begin(), own.end());
            olow.insert(olow.end(), M.k.begin(), M.k.end());
            bool use_own = false;
            if (T.producer >= 0) {
                const Merge &Pm = P.merges[size_t(T.producer)];
                std::set<int> tiled(Pm.m.begin(), Pm.m.end());
                tiled.insert(Pm.n.begin(), Pm.n.end());
                auto lead = [&](const std::vector<int> &v) {
                    size_t c = 0;
                    while (c < v.size() && tiled.count(v[c])) ++c;
                    return c;
                };
                use_own = lead(olow) > lead(klow);
            }
            T.own_low = use_own;
            T.layout = use_own ? olow : klow;
            T.layout.insert(T.layout.end(), M.b.begin(), M.b.end());
        };
        lay(P.tens[M.x], M.m);
        lay(P.tens[M.y], M.n);
    }
    return QS_OK;
}

// The greedy order is tried kTrials times with different tie-breaks (trial 0:
// lowest vertex first); the plan with the fewest flops is kept.
constexpr int kTrials = 16;

qs_status make_plan_uncached(const qs_circuit *c, int n, int nslice, Plan &P)
{
    Plan G;
    if (qs_status st = build_graph(c, n, nslice, G)) return st;
    qs_status last = QS_OK;
    bool have = false;
    for (int trial = 0; trial < kTrials; ++trial) {
        Plan T = G;
        if (qs_status st = plan_merges(T, trial)) {
            last = st;
            continue;
        }
        const double f = T.flops0 + T.flops1 * std::ldexp(1.0, T.nslice);
        if (!have || f < P.flops0 + P.flops1 * std::ldexp(1.0, P.nslice)) {
            P = std::move(T);
            have = true;
        }
    }
    return have ? QS_OK : last;
}

// Plans are kept with the circuit, per (n, nslice), until it changes.
qs_status make_plan(const qs_circuit *c, int n, int nslice, std::shared_ptr<const Plan> &out)
{
    if (!c) return sfail(QS_E_INVAL, "circuit is NULL");
    const uint64_t key = (uint64_t(0x5A) << 56) | (uint64_t(uint32_t(n)) << 8) | uint64_t(uint8_t(nslice));
    if (n >= 1 && n <= QS_MAX_CIRCUIT_QUBITS && nslice >= 0 && nslice <= QS_SINGLE_MAX_SLICES)
        if (auto v = qs::circuit_cache_get(c, key)) {
            out = std::static_pointer_cast<const Plan>(v);
            return QS_OK;
        }
    auto P = std::make_shared<Plan>();
    if (qs_status st = make_plan_uncached(c, n, nslice, *P)) return st;
    qs::circuit_cache_put(c, key, P);
    out = P;
    return QS_OK;
}

// ------------------------------------------------------------ memory plan --

size_t ten_bytes(const Ten &t, uint32_t bt) { return (size_t(16) << t.idx.size()) * (t.batched ? bt : 1); }

// First-fit placement of every tensor in one arena: initial tensors at the
// start, each merge's result before its operands are released.
size_t place(const Plan &P, uint32_t bt, std::vector<size_t> &off)
{
    off.assign(P.tens.size(), 0);
    std::map<size_t, size_t> freel;  // offset -> length of free gaps below `top`
    size_t top = 0, peak = 0;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    auto alloc = [&](size_t len) {
        len = up(len);
        for (auto it = freel.begin(); it != freel.end(); ++it)
            if (it->second >= len) {
                const size_t o = it->first, rest = it->second - len;
                freel.erase(it);
                if (rest) freel[o + len] = rest;
                return o;
            }
        const size_t o = top;
        top += len;
        peak = std::max(peak, top);
        return o;
    };
    auto release = [&](size_t o, size_t len) {
        len = up(len);
        auto it = freel.emplace(o, len).first;
        auto nx = std::next(it);  // coalesce with the gap above
        if (nx != freel.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            freel.erase(nx);
        }
        if (it != freel.begin()) {  // and with the gap below
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                freel.erase(it);
            }
        }
    };
    for (size_t t = 0; t < P.tens.size(); ++t)
        if (P.tens[t].base >= 0) off[t] = alloc(ten_bytes(P.tens[t], bt));
    for (const Merge &M : P.merges) {
        off[M.z] = alloc(ten_bytes(P.tens[M.z], bt));
        release(off[M.x], ten_bytes(P.tens[M.x], bt));
        release(off[M.y], ten_bytes(P.tens[M.y], bt));
    }
    return peak;
}

void fill_info(const Plan &P, uint32_t bt, size_t peak, qs_single_info *info)
{
    if (!info) return;
    info->vertices = int(P.verts.size());
    info->tensors = int(P.tens.size() - P.merges.size());
    info->fixed = P.fixed;
    info->sliced = P.nslice;
    info->merges = int(P.merges.size());
    info->max_rank = P.max_rank;
    info->flops = P.flops0 + P.flops1 * std::ldexp(1.0, P.nslice);
    info->peak_bytes = double(peak);
    info->batch = int(bt);
    info->own_low = 0;
    for (const Ten &t : P.tens) info->own_low += t.own_low;
}

constexpr double kSingleBudget = 64.0 * (1ull << 30);  // device arena of one call, at most

}  // namespace

extern "C" {

qs_status qs_single_plan(const qs_circuit *c, int n, int nslice, qs_single_info *info)
try {
    std::shared_ptr<const Plan> PP;
    if (qs_status st = make_plan(c, n, nslice, PP)) return st;
    const Plan &P = *PP;
    std::vector<size_t> off;
    const uint32_t bt = uint32_t(1) << P.nslice;
    fill_info(P, bt, place(P, bt, off), info);
    return QS_OK;
} catch (const std::bad_alloc &) {
    return sfail(QS_E_NOMEM, "host allocation failed while planning the contraction");
}

qs_status qs_single_amplitudes(const qs_circuit *c, int n, const uint64_t *bits, size_t m, int nslice, double *out,
                               qs_single_info *info)
try {
    if (m && (!bits || !out)) return sfail(QS_E_INVAL, "bits or out is NULL");
    std::shared_ptr<const Plan> PP;
    if (qs_status st = make_plan(c, n, nslice, PP)) return st;
    const Plan &P = *PP;
    for (size_t w = 0; w < m; ++w)
        if (n < 64 && (bits[w] >> n)) return sfail(QS_E_RANGE, "bitstring %zu sets a qubit >= %d", w, n);
    const uint32_t S = uint32_t(1) << P.nslice;
    std::vector<size_t> off;
    const size_t peak1 = place(P, S, off);
    const size_t lim = qs::memory_limit();
    const double budget = lim ? std::min(kSingleBudget, double(lim)) : kSingleBudget;
    if (double(peak1) > budget)
        return sfail(QS_E_NOMEM, "the contraction needs %.1f GiB for one bitstring", double(peak1) / (1ull << 30));
    // bitstrings per chunk: the batched tensors grow with it
    size_t words = std::max<size_t>(1, size_t(budget / std::max<double>(double(peak1), 1.0)));
    words = std::min<size_t>({words, m ? m : 1, size_t(1) << 16, size_t(UINT32_MAX / S)});
    fill_info(P, uint32_t(words) * S, 0, info);
    if (m == 0) return QS_OK;
    hipStream_t st = nullptr;
    void *arena = nullptr, *bases = nullptr, *aux = nullptr;
    auto cleanup = [&](qs_status r) {
        if (st) (void)hipStreamSynchronize(st);
        if (arena) (void)hipFree(arena);
        if (bases) (void)hipFree(bases);
        if (aux) (void)hipFree(aux);
        if (st) (void)hipStreamDestroy(st);
        return r;
    };
    auto hfail = [&](hipError_t e, const char *what) {
        return cleanup(e == hipErrorOutOfMemory ? sfail(QS_E_NOMEM, "%s: out of device memory", what)
                                                : sfail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e)));
    };
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        st = nullptr;
        return hfail(e, "stream creation");
    }
    // every gate tensor, uploaded once
    std::vector<size_t> boff(P.bases.size());
    size_t btotal = 0;
    for (size_t i = 0; i < P.bases.size(); ++i) {
        boff[i] = btotal;
        btotal += P.bases[i].v.size() * 16;
    }
    std::vector<double> hb(btotal / 8);
    for (size_t i = 0; i < P.bases.size(); ++i)
        std::memcpy(hb.data() + boff[i] / 8, P.bases[i].v.data(), P.bases[i].v.size() * 16);
    if ((e = hipMalloc(&bases, std::max<size_t>(btotal, 16))) != hipSuccess) return hfail(e, "gate tensors");
    if ((e = hipMemcpyAsync(bases, hb.data(), btotal, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hfail(e, "gate tensors");
    const size_t nf = P.finals.size();
    const size_t aux_bytes = words * 8 + words * 16 + nf * 16 + 256;
    if ((e = hipMalloc(&aux, aux_bytes)) != hipSuccess) return hfail(e, "single-amplitude buffers");
    uint64_t *dbits = static_cast<uint64_t *>(aux);
    double2 *dout = reinterpret_cast<double2 *>(static_cast<char *>(aux) + words * 8);
    const double2 **dscal = reinterpret_cast<const double2 **>(static_cast<char *>(aux) + words * 24);
    uint64_t *dstr = reinterpret_cast<uint64_t *>(static_cast<char *>(aux) + words * 24 + nf * 8);
    size_t arena_bytes = 0;
    for (size_t w0 = 0; w0 < m; w0 += words) {
        const uint32_t cw = uint32_t(std::min(words, m - w0));
        const uint32_t bt = cw * S;
        const size_t need = place(P, bt, off);
        if (need > arena_bytes) {
            if (arena) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(arena);
                arena = nullptr;
            }
            if ((e = hipMalloc(&arena, std::max<size_t>(need, 256))) != hipSuccess) return hfail(e, "tensor arena");
            arena_bytes = need;
        }
        char *A = static_cast<char *>(arena);
        auto dptr = [&](int t) { return reinterpret_cast<double2 *>(A + off[t]); };
        if ((e = hipMemcpyAsync(dbits, bits + w0, cw * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hfail(e, "bitstrings");
        // initial tensors, fixed vertices substituted, in their consumers' order
        for (size_t t = 0; t < P.tens.size(); ++t) {
            const Ten &T = P.tens[t];
            if (T.base < 0) continue;
            const Base &B = P.bases[T.base];
            qs::SaPrep p{};
            p.base = reinterpret_cast<const double2 *>(static_cast<char *>(bases) + boff[T.base]);
            p.out = dptr(int(t));
            p.nbt = T.batched ? bt : 1;
            p.so = T.batched ? (uint64_t(1) << T.idx.size()) : 0;
            p.slices = S;
            p.r = int(T.idx.size());
            const std::vector<int> &L = T.layout.empty() ? T.idx : T.layout;
            for (int q = 0; q < p.r; ++q)
                p.src[q] = uint8_t(std::find(B.idx.begin(), B.idx.end(), L[q]) - B.idx.begin());
            for (size_t j = 0; j < B.idx.size(); ++j) {
                const Vert &V = P.verts[B.idx[j]];
                if (V.kind == V_FREE) continue;
                p.fpos[p.nf] = uint8_t(j);
                p.fkind[p.nf] = uint8_t(V.kind == V_INPUT ? 0 : (V.kind == V_OUTPUT ? 1 : 2));
                p.fwhich[p.nf] = uint8_t(V.which);
                ++p.nf;
            }
            if ((e = qs::launch_sa_prep(p, dbits, st)) != hipSuccess) return hfail(e, "tensor placement");
        }
        // the eliminations
        for (const Merge &M : P.merges) {
            const Ten &X = P.tens[M.x], &Y = P.tens[M.y], &Z = P.tens[M.z];
            qs::SaContract k{};
            k.x = dptr(M.x);
            k.y = dptr(M.y);
            k.z = dptr(M.z);
            k.sx = X.batched ? (uint64_t(1) << X.idx.size()) : 0;
            k.sy = Y.batched ? (uint64_t(1) << Y.idx.size()) : 0;
            k.sz = Z.batched ? (uint64_t(1) << Z.idx.size()) : 0;
            k.nbt = Z.batched ? bt : 1;
            k.nb = int(M.b.size());
            k.nm = int(M.m.size());
            k.nn = int(M.n.size());
            k.nk = int(M.k.size());
            k.xo = X.own_low ? 1 : 0;
            k.yo = Y.own_low ? 1 : 0;
            const std::vector<int> &L = Z.layout.empty() ? Z.idx : Z.layout;
            auto pos = [&](int v) { return uint8_t(std::find(L.begin(), L.end(), v) - L.begin()); };
            for (int j = 0; j < k.nb; ++j) k.pb[j] = pos(M.b[j]);
            for (int j = 0; j < k.nm; ++j) k.pm[j] = pos(M.m[j]);
            for (int j = 0; j < k.nn; ++j) k.pn[j] = pos(M.n[j]);
            for (int j = 0; j < k.nb; ++j) k.bfast |= k.pb[j] == 0;
            const double outs = double(k.nbt) * std::ldexp(1.0, k.nb + k.nm + k.nn);
            int kern = qs::SA_THREAD;
            if (k.nm >= 6 && k.nn >= 6 && k.nk >= 3)
                kern = qs::SA_TILE;
            else if (k.nk >= 5 && outs < double(1 << 22))
                kern = qs::SA_WAVE;
            if ((e = qs::launch_sa_contract(k, kern, st)) != hipSuccess) return hfail(e, "tensor merge");
        }
        // product of the scalars per graph, summed over the graphs
        std::vector<const double2 *> sp(nf);
        std::vector<uint64_t> ss(nf);
        for (size_t i = 0; i < nf; ++i) {
            sp[i] = dptr(P.finals[i]);
            ss[i] = P.tens[P.finals[i]].batched ? 1 : 0;
        }
        if (nf) {
            if ((e = hipMemcpyAsync(dscal, sp.data(), nf * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = hipMemcpyAsync(dstr, ss.data(), nf * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
                return hfail(e, "scalars");
        }
        if ((e = qs::launch_sa_finish(dscal, dstr, int(nf), cw, S, dbits, P.idle, dout, st)) != hipSuccess)
            return hfail(e, "amplitude sum");
        if ((e = hipMemcpyAsync(out + 2 * w0, dout, cw * 16, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hfail(e, "amplitudes");
    }
    fill_info(P, uint32_t(words) * S, arena_bytes, info);
    return cleanup(QS_OK);
} catch (const std::bad_alloc &) {
    return sfail(QS_E_NOMEM, "host allocation failed in the single-amplitude mode");
}

}  // extern "C"
