// Group expansion, gate canonicalisation, greedy fusion and the trajectory
// runner (host side of libqs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <thread>
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
// Complex products are written out (std::complex products go through the
// C99 NaN-recovering multiply, which dominates planning time otherwise).
void apply_local(std::vector<cd> &M, int k, const std::vector<int> &tbits,
                 const std::vector<int> &cbits, const std::vector<double> &m)
{
    const int D = 1 << k;
    const int nt = int(tbits.size());
    const int g = 1 << nt;
    int tmask = 0, cmask = 0;
    for (int b : tbits) tmask |= 1 << b;
    for (int b : cbits) cmask |= 1 << b;
    int off[64];
    for (int x = 0; x < g; ++x) {
        int o = 0;
        for (int b = 0; b < nt; ++b)
            if ((x >> (nt - 1 - b)) & 1) o |= 1 << tbits[b];
        off[x] = o;
    }
    double v[128], w[128];
    for (int i = 0; i < D; ++i) {
        if ((i & tmask) || (i & cmask) != cmask) continue;
        for (int col = 0; col < D; ++col) {
            for (int x = 0; x < g; ++x) {
                const cd a = M[size_t(i | off[x]) * D + col];
                v[2 * x] = a.real();
                v[2 * x + 1] = a.imag();
            }
            for (int r = 0; r < g; ++r) {
                double re = 0.0, im = 0.0;
                const double *mr = m.data() + size_t(2) * r * g;
                for (int c = 0; c < g; ++c) {
                    re += mr[2 * c] * v[2 * c] - mr[2 * c + 1] * v[2 * c + 1];
                    im += mr[2 * c] * v[2 * c + 1] + mr[2 * c + 1] * v[2 * c];
                }
                w[2 * r] = re;
                w[2 * r + 1] = im;
            }
            for (int x = 0; x < g; ++x) M[size_t(i | off[x]) * D + col] = cd(w[2 * x], w[2 * x + 1]);
        }
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

int default_tile_qubits(int n) { return n < 13 ? n : 13; }

int default_kmax(int n, qs_dtype dt)
{
    (void)n;
    (void)dt;
    return 3;
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

// ======================================================== tile planning ==

namespace qs {

namespace {

struct GInfo {
    CanonGate c;
    uint64_t qmask = 0;  // targets | controls
    uint64_t tmask = 0;  // targets
    uint64_t cmask = 0;  // controls
    bool diag = false;
    bool logical = true;
};

uint64_t mask_of(const std::vector<int> &v)
{
    uint64_t m = 0;
    for (int q : v) m |= uint64_t(1) << q;
    return m;
}

std::vector<int> bits_desc(uint64_t m)
{
    std::vector<int> v;
    for (int q = 63; q >= 0; --q)
        if (m >> q & 1) v.push_back(q);
    return v;
}

bool is_diag_matrix(const std::vector<double> &m, int k)
{
    const int D = 1 << k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if (r != c && (m[2 * (r * D + c)] != 0.0 || m[2 * (r * D + c) + 1] != 0.0)) return false;
    return true;
}

struct OpenBlock {
    uint64_t qmask = 0;  // qubits inside the tile
    uint64_t omask = 0;  // qubits outside the tile (constant per tile)
    std::vector<const GInfo *> gates;
};

// A gate of a block in block-local terms.  Qubit sources are a local bit
// (>= 0) or an outer selector slot s encoded as ~s.
struct LocalGate {
    bool diag = false;
    int tmask = 0, cmask = 0;     // dense: local target / inner control masks
    int g = 1;                    // dense: 2^targets
    int off[64];                  // dense: local offset of target pattern x (targets[0] = MSB)
    std::vector<int> octl;        // dense: outer slots that must be 1
    std::vector<int> tsrc, csrc;  // diagonal: sources of the table index bits and of the controls
    int reads = 0;                // outer slots the gate depends on (bit s)
    const double *m = nullptr;    // dense matrix or diagonal table
};

// Left-multiply the block matrix M (D x D, row-major, interleaved complex)
// by one block-local gate with the outer slots set to `oval`.
void apply_local_gate(double *M, int D, const LocalGate &L, const int *oval)
{
    const size_t rs = size_t(2) * D;
    if (L.diag) {
        for (int i = 0; i < D; ++i) {
            bool on = true;
            for (int s : L.csrc)
                if (!(s >= 0 ? (i >> s) & 1 : oval[~s])) {
                    on = false;
                    break;
                }
            if (!on) continue;
            int x = 0;
            for (int s : L.tsrc) x = (x << 1) | (s >= 0 ? (i >> s) & 1 : oval[~s]);
            const double fr = L.m[2 * x], fi = L.m[2 * x + 1];
            if (fr == 1.0 && fi == 0.0) continue;
            double *row = M + rs * i;
            for (int c = 0; c < D; ++c) {
                const double a = row[2 * c], b = row[2 * c + 1];
                row[2 * c] = a * fr - b * fi;
                row[2 * c + 1] = a * fi + b * fr;
            }
        }
        return;
    }
    for (int s : L.octl)
        if (!oval[s]) return;
    const double *m = L.m;
    if (L.g == 2) {
        const double m00r = m[0], m00i = m[1], m01r = m[2], m01i = m[3];
        const double m10r = m[4], m10i = m[5], m11r = m[6], m11i = m[7];
        for (int i = 0; i < D; ++i) {
            if ((i & L.tmask) || (i & L.cmask) != L.cmask) continue;
            double *a = M + rs * i, *b = M + rs * (i | L.off[1]);
            for (int c = 0; c < D; ++c) {
                const double ar = a[2 * c], ai = a[2 * c + 1], br = b[2 * c], bi = b[2 * c + 1];
                a[2 * c] = m00r * ar - m00i * ai + m01r * br - m01i * bi;
                a[2 * c + 1] = m00r * ai + m00i * ar + m01r * bi + m01i * br;
                b[2 * c] = m10r * ar - m10i * ai + m11r * br - m11i * bi;
                b[2 * c + 1] = m10r * ai + m10i * ar + m11r * bi + m11i * br;
            }
        }
        return;
    }
    double v[128], w[128];
    for (int i = 0; i < D; ++i) {
        if ((i & L.tmask) || (i & L.cmask) != L.cmask) continue;
        for (int col = 0; col < D; ++col) {
            for (int x = 0; x < L.g; ++x) {
                const double *a = M + rs * (i | L.off[x]) + 2 * col;
                v[2 * x] = a[0];
                v[2 * x + 1] = a[1];
            }
            for (int r = 0; r < L.g; ++r) {
                double re = 0.0, im = 0.0;
                const double *mr = m + size_t(2) * r * L.g;
                for (int c = 0; c < L.g; ++c) {
                    re += mr[2 * c] * v[2 * c] - mr[2 * c + 1] * v[2 * c + 1];
                    im += mr[2 * c] * v[2 * c + 1] + mr[2 * c + 1] * v[2 * c];
                }
                w[2 * r] = re;
                w[2 * r + 1] = im;
            }
            for (int x = 0; x < L.g; ++x) {
                double *a = M + rs * (i | L.off[x]) + 2 * col;
                a[0] = w[2 * x];
                a[1] = w[2 * x + 1];
            }
        }
    }
}

// Block matrices over the tile qubits `qs` (qs[0] = MSB) for every assignment
// p of the outer qubits `os` (bit |os|-1-b of p = value of os[b]):
// mats[which[p]] is the matrix of pattern p.
void block_matrices(const std::vector<int> &qs, const std::vector<int> &os,
                    const std::vector<const GInfo *> &gates, std::vector<std::vector<double>> &mats,
                    std::vector<int> &which)
{
    const int k = int(qs.size()), D = 1 << k, no = int(os.size()), P = 1 << no;
    int lbit[64], oslot[64];
    for (int q = 0; q < 64; ++q) lbit[q] = oslot[q] = -1;
    for (int i = 0; i < k; ++i) lbit[qs[i]] = k - 1 - i;
    for (int b = 0; b < no; ++b) oslot[os[b]] = b;
    auto src = [&](int q) { return lbit[q] >= 0 ? lbit[q] : ~oslot[q]; };
    std::vector<LocalGate> lg(gates.size());
    for (size_t j = 0; j < gates.size(); ++j) {
        const CanonGate &c = gates[j]->c;
        LocalGate &L = lg[j];
        L.m = c.m.data();
        if (c.kind == CanonGate::PHASE) {
            L.diag = true;
            for (int q : c.targets) L.tsrc.push_back(src(q));
            for (int q : c.controls) L.csrc.push_back(src(q));
            for (int s : L.tsrc)
                if (s < 0) L.reads |= 1 << ~s;
            for (int s : L.csrc)
                if (s < 0) L.reads |= 1 << ~s;
            continue;
        }
        const int nt = int(c.targets.size());
        L.g = 1 << nt;
        for (int q : c.targets) L.tmask |= 1 << lbit[q];
        for (int x = 0; x < L.g; ++x) {
            int o = 0;
            for (int b = 0; b < nt; ++b)
                if ((x >> (nt - 1 - b)) & 1) o |= 1 << lbit[c.targets[b]];
            L.off[x] = o;
        }
        for (int q : c.controls) {
            if (lbit[q] >= 0) {
                L.cmask |= 1 << lbit[q];
            } else {
                L.octl.push_back(oslot[q]);
                L.reads |= 1 << oslot[q];
            }
        }
    }
    // Gates run in order on a list of partial products, one per assignment
    // of the outer bits read so far; a gate that reads a new outer bit first
    // splits every entry of the list.  Patterns differing only in bits no
    // gate reads share a product.
    struct Live {
        int vals;  // values of the assigned outer slots (bit s)
        std::vector<double> M;
    };
    std::vector<Live> live(1);
    live[0].vals = 0;
    live[0].M.assign(size_t(2) * D * D, 0.0);
    for (int i = 0; i < D; ++i) live[0].M[2 * (size_t(i) * D + i)] = 1.0;
    int assigned = 0;
    int oval[64];
    for (const LocalGate &L : lg) {
        const int fresh = L.reads & ~assigned;
        for (int b = 0; b < no; ++b) {
            if (!(fresh >> b & 1)) continue;
            const size_t cnt = live.size();
            for (size_t u = 0; u < cnt; ++u) {
                Live one = live[u];
                one.vals |= 1 << b;
                live.push_back(std::move(one));
            }
        }
        assigned |= fresh;
        for (Live &e : live) {
            for (int b = 0; b < no; ++b) oval[b] = e.vals >> b & 1;
            apply_local_gate(e.M.data(), D, L, oval);
        }
    }
    mats.clear();
    which.assign(P, 0);
    for (int p = 0; p < P; ++p) {
        int v = 0;
        for (int b = 0; b < no; ++b) v |= ((p >> (no - 1 - b)) & 1) << b;
        v &= assigned;
        for (size_t u = 0; u < live.size(); ++u)
            if (live[u].vals == v) {
                which[p] = int(u);
                break;
            }
    }
    for (Live &e : live) mats.push_back(std::move(e.M));
}

}  // namespace

namespace {

void plan_tiles_once(const std::vector<FlatOp> &flat, size_t k0, size_t e, int n, const TileParams &tp,
                     std::vector<PlanStep> &out)
{
    const int m = std::min(tp.m, n);
    const int L = std::min(tp.L, m);
    const int kmax = std::min(tp.kmax, m);
    const int mo = std::max(0, std::min(tp.max_outer, kMaxOuter));
    std::vector<GInfo> info;
    info.reserve(e - k0);
    for (size_t i = k0; i < e; ++i) {
        const FlatOp &f = flat[i];
        GInfo g;
        g.c = canonicalize(f.targets.data(), int(f.targets.size()), f.controls.data(),
                           int(f.controls.size()), f.m.data());
        if (g.c.kind == CanonGate::IDENTITY) continue;
        g.tmask = mask_of(g.c.targets);
        g.cmask = mask_of(g.c.controls);
        g.qmask = g.tmask | g.cmask;
        g.diag = g.c.kind == CanonGate::PHASE;
        info.push_back(std::move(g));
    }
    const uint64_t low = (L >= 64) ? ~uint64_t(0) : ((uint64_t(1) << L) - 1);
    std::vector<size_t> remaining(info.size());
    for (size_t i = 0; i < info.size(); ++i) remaining[i] = i;
    auto fits_tile = [&](const GInfo &g) {
        // a gate can live in a tile when its qubits inside any Q are few
        // enough: dense gates need all targets in Q and at most kmax local
        // qubits; diagonal gates at most 3 local and 3 outer qubits (table)
        if (g.diag) return __builtin_popcountll(g.qmask) <= kmax + mo;
        return __builtin_popcountll(g.tmask) <= kmax && __builtin_popcountll(g.cmask) <= kmax + mo;
    };
    while (!remaining.empty()) {
        // ---- choose Q and the gates this sweep applies
        uint64_t Q = low;
        uint64_t blocked = 0;
        std::vector<size_t> applied, deferred;
        for (size_t gi : remaining) {
            const GInfo &g = info[gi];
            if ((g.qmask & blocked) || !fits_tile(g)) {
                deferred.push_back(gi);
                blocked |= g.qmask;
                continue;
            }
            if (g.diag) {
                // at most `mo` of its qubits may stay outside the tile
                int extra = __builtin_popcountll(g.qmask & ~Q) - mo;
                if (extra > 0 && __builtin_popcountll(Q) + extra <= m) {
                    for (uint64_t r = g.qmask & ~Q; extra > 0; r &= r - 1, --extra) Q |= r & (~r + 1);
                }
                applied.push_back(gi);
                continue;
            }
            const uint64_t need = g.tmask & ~Q;
            if (!need || __builtin_popcountll(Q | need) <= m) {
                Q |= need;
                applied.push_back(gi);
                continue;
            }
            deferred.push_back(gi);
            blocked |= g.qmask;
        }
        if (applied.empty()) {
            // the first gate does not fit any tile: apply it on its own
            PlanStep st;
            st.sweep = false;
            st.gate = info[remaining[0]].c;
            out.push_back(std::move(st));
            remaining.erase(remaining.begin());
            continue;
        }
        for (int q = 0; q < n && __builtin_popcountll(Q) < m; ++q) Q |= uint64_t(1) << q;
        if (tp.search) {
            // Local search over the tile qubits: the greedy set takes the
            // qubits of the earliest pending gates, which on layered circuits
            // leaves many of a sweep's gates blocked by a neighbour outside the
            // tile.  From the greedy set and from `restarts` random sets, swap
            // one qubit of Q (never the L lowest) for one outside whenever the
            // sweep then applies more gates, until no swap helps.  Among the
            // local optima keep the one whose sweep plus the next sweep (its
            // deferred gates, searched the same way from their greedy set),
            // and so on up to `lookahead` sweeps, apply the most gates; ties
            // keep the earliest candidate.  Counts
            // come from the scan below with Q fixed, post-pass rules
            // included, so the chosen Q's lists come from the same scan.
            auto scan_on = [&](const std::vector<size_t> &rem, uint64_t Qf, std::vector<size_t> *app,
                               std::vector<size_t> *def) {
                uint64_t blk = 0;
                int c = 0;
                for (size_t gi : rem) {
                    const GInfo &g = info[gi];
                    const bool ok = !(g.qmask & blk) && fits_tile(g) && (g.diag || !(g.tmask & ~Qf)) &&
                                    __builtin_popcountll(g.qmask & Qf) <= kmax &&
                                    __builtin_popcountll(g.qmask & ~Qf) <= mo;
                    if (ok) {
                        ++c;
                        if (app) app->push_back(gi);
                    } else {
                        blk |= g.qmask;
                        if (def) def->push_back(gi);
                    }
                }
                return c;
            };
            // with a run weight, a tile set whose lowest 5 or 6 qubits are
            // contiguous (rows of 256 or 512 bytes instead of 128) counts
            // that many gates more per extra qubit
            auto run_bonus = [&](uint64_t q) {
                const int run = __builtin_ctzll(~q);
                return tp.run_weight * std::min(2, std::max(0, run - 4));
            };
            auto climb = [&](const std::vector<size_t> &rem, uint64_t Qs, int &count) {
                int best = scan_on(rem, Qs, nullptr, nullptr) + run_bonus(Qs);
                for (bool improved = true; improved;) {
                    improved = false;
                    for (int a = L; a < n && !improved; ++a) {
                        if (!(Qs >> a & 1)) continue;
                        for (int b = L; b < n; ++b) {
                            if (Qs >> b & 1) continue;
                            const uint64_t Q2 = (Qs & ~(uint64_t(1) << a)) | (uint64_t(1) << b);
                            const int c2 = scan_on(rem, Q2, nullptr, nullptr) + run_bonus(Q2);
                            if (c2 > best) {
                                best = c2;
                                Qs = Q2;
                                improved = true;
                                break;
                            }
                        }
                    }
                }
                count = best;
                return Qs;
            };
            // first-come tile qubits of a gate list (the start of the next
            // sweep's search)
            auto greedy_q = [&](const std::vector<size_t> &rem) {
                uint64_t Qg = low, blk = 0;
                for (size_t gi : rem) {
                    const GInfo &g = info[gi];
                    if ((g.qmask & blk) || !fits_tile(g)) {
                        blk |= g.qmask;
                        continue;
                    }
                    if (g.diag) continue;
                    const uint64_t need = g.tmask & ~Qg;
                    if (!need || __builtin_popcountll(Qg | need) <= m)
                        Qg |= need;
                    else
                        blk |= g.qmask;
                }
                for (int q = 0; q < n && __builtin_popcountll(Qg) < m; ++q) Qg |= uint64_t(1) << q;
                return Qg;
            };
            std::vector<std::pair<uint64_t, int>> cands;
            {
                int c = 0;
                const uint64_t q0 = climb(remaining, Q, c);
                cands.push_back({q0, c});
            }
            uint64_t rs = 0x9E3779B97F4A7C15ull ^ (uint64_t(out.size()) << 17);  // xorshift64, per sweep
            for (int r = 0; r < tp.restarts && n - L > m - L; ++r) {
                uint64_t Qr = low;
                while (__builtin_popcountll(Qr) < m) {
                    rs ^= rs << 13;
                    rs ^= rs >> 7;
                    rs ^= rs << 17;
                    Qr |= uint64_t(1) << (L + int(rs % uint64_t(n - L)));
                }
                int c = 0;
                const uint64_t qc = climb(remaining, Qr, c);
                bool seen = false;
                for (auto &x : cands) seen = seen || x.first == qc;
                if (!seen) cands.push_back({qc, c});
            }
            size_t bi = 0;
            int bscore = -1;
            for (size_t ci = 0; ci < cands.size(); ++ci) {
                int score = cands[ci].second;
                if (cands.size() > 1) {
                    std::vector<size_t> app, def;
                    scan_on(remaining, cands[ci].first, &app, &def);
                    // the following sweeps, each from its greedy set
                    for (int l = 2; l <= tp.lookahead && !def.empty(); ++l) {
                        int cl = 0;
                        const uint64_t ql = climb(def, greedy_q(def), cl);
                        score += cl;
                        if (l == tp.lookahead) break;
                        std::vector<size_t> a2, d2;
                        scan_on(def, ql, &a2, &d2);
                        def.swap(d2);
                    }
                }
                if (score > bscore) {
                    bscore = score;
                    bi = ci;
                }
            }
            Q = cands[bi].first;
            applied.clear();
            deferred.clear();
            scan_on(remaining, Q, &applied, &deferred);
        }
        // gates with more than kmax qubits inside or `mo` outside the final Q
        // are left for a later step
        {
            std::vector<size_t> keep;
            uint64_t blk = 0;
            std::vector<size_t> later;
            for (size_t gi : applied) {
                const GInfo &g = info[gi];
                const bool bad = __builtin_popcountll(g.qmask & Q) > kmax ||
                                 __builtin_popcountll(g.qmask & ~Q) > mo;
                if (bad || (g.qmask & blk)) {
                    later.push_back(gi);
                    blk |= g.qmask;
                } else {
                    keep.push_back(gi);
                }
            }
            if (!later.empty()) {
                // re-merge into circuit order with the deferred gates
                std::vector<size_t> rest = later;
                rest.insert(rest.end(), deferred.begin(), deferred.end());
                std::sort(rest.begin(), rest.end());
                deferred.swap(rest);
                applied.swap(keep);
            }
        }
        if (applied.empty()) {
            // nothing left for this tile: the first gate goes on its own
            PlanStep st;
            st.sweep = false;
            st.gate = info[remaining[0]].c;
            out.push_back(std::move(st));
            remaining.erase(remaining.begin());
            continue;
        }
        // ---- fuse the applied gates into tile ops
        Sweep sw;
        for (int q = 0; q < 64; ++q)
            if (Q >> q & 1) sw.Q.push_back(q);
        sw.gates = int(applied.size());
        std::vector<std::vector<double>> mats;
        std::vector<int> which;
        auto emit_block = [&](OpenBlock &b) {
            const std::vector<int> os = bits_desc(b.omask);
            const int P = 1 << os.size();
            const std::vector<int> qs = bits_desc(b.qmask);
            TileOp op;
            op.outer = os;
            if (qs.size() <= 3) {
                // narrow blocks that are diagonal for every outer pattern
                block_matrices(qs, os, b.gates, mats, which);
                bool all_diag = true;
                for (auto &mm : mats) all_diag = all_diag && is_diag_matrix(mm, int(qs.size()));
                if (all_diag) {
                    op.kind = TileOp::PHASE;
                    op.qubits = qs;
                    const int D = 1 << qs.size();
                    op.m.resize(size_t(2) * D * P);
                    for (int p = 0; p < P; ++p) {
                        const std::vector<double> &mp = mats[which[p]];
                        for (int x = 0; x < D; ++x) {
                            op.m[2 * (p * D + x)] = mp[2 * (x * D + x)];
                            op.m[2 * (p * D + x) + 1] = mp[2 * (x * D + x) + 1];
                        }
                    }
                    sw.ops.push_back(std::move(op));
                    return;
                }
            }
            uint64_t pm = b.qmask;
            // widen narrow blocks to the 4-qubit matrix-core shape with
            // identity factors on otherwise untouched tile qubits
            for (int q : sw.Q) {
                if (__builtin_popcountll(pm) >= 4) break;
                pm |= uint64_t(1) << q;
            }
            op.kind = TileOp::DENSE;
            op.qubits = bits_desc(pm);
            const int k = int(op.qubits.size());
            block_matrices(op.qubits, os, b.gates, mats, which);
            std::vector<char> ident(mats.size());
            for (size_t u = 0; u < mats.size(); ++u) {
                ident[u] = is_identity(mats[u], k);
                op.m.insert(op.m.end(), mats[u].begin(), mats[u].end());
            }
            op.pmap.resize(P);
            for (int p = 0; p < P; ++p) {
                op.pmap[p] = uint8_t(which[p]);
                if (ident[which[p]]) op.skip |= 1u << p;
            }
            sw.ops.push_back(std::move(op));
        };
        // Blocks by a light-cone scan: open a block at the first remaining
        // gate and absorb, in circuit order, every later gate whose tile
        // qubits keep the block within kmax (and its outer selectors within
        // max_outer), skipping gates that touch a qubit of an earlier skipped
        // gate.
        // Skipped gates do not precede absorbed ones on a shared tile qubit,
        // and outer qubits are constant over the sweep, so the absorbed
        // gates may run first.
        std::vector<size_t> rem = applied;
        while (!rem.empty()) {
            OpenBlock blk;
            uint64_t blocked = 0;
            std::vector<size_t> rest;
            for (size_t gi : rem) {
                const GInfo &g = info[gi];
                const uint64_t loc = g.qmask & Q, outm = g.qmask & ~Q;
                if (loc & blocked) {
                    rest.push_back(gi);
                    blocked |= loc;
                    continue;
                }
                const uint64_t uni = blk.qmask | loc, ouni = blk.omask | outm;
                if (__builtin_popcountll(uni) <= kmax && __builtin_popcountll(ouni) <= mo) {
                    blk.qmask = uni;
                    blk.omask = ouni;
                    blk.gates.push_back(&g);
                } else {
                    rest.push_back(gi);
                    blocked |= loc;
                }
            }
            emit_block(blk);
            rem.swap(rest);
        }
        PlanStep st;
        st.sweep = true;
        st.sw = std::move(sw);
        out.push_back(std::move(st));
        remaining.swap(deferred);
    }
}

}  // namespace

// Relative cost of a tiled plan: a sweep costs its memory pass (1; 0.975
// when the tile holds qubits 0..4, 0.925 with 0..5: rows of 256 and 512
// bytes against 128 move faster, 0.975 and 0.89 on the tile microbenchmark
// with four ops, and 0.925 fits the whole plans measured) plus 0.15 per dense
// block beyond the two that hide under that pass, a gate applied on its own
// one pass.  The ratio is the per-op time of the tile kernel beyond the
// second op over its memory time (0.37 over 3.75 ms on the microbenchmark,
// 0.11-0.15 in whole plans of 30- and 34-qubit circuits).
double plan_cost(const std::vector<PlanStep> &steps)
{
    double c = 0;
    for (const PlanStep &st : steps) {
        if (!st.sweep) {
            c += 1;
            continue;
        }
        int dense = 0;
        for (const TileOp &op : st.sw.ops) dense += op.kind == TileOp::DENSE;
        int run = 0;
        while (run < int(st.sw.Q.size()) && st.sw.Q[run] == run) ++run;
        c += (run >= 6 ? 0.925 : run == 5 ? 0.975 : 1.0) + 0.15 * std::max(0, dense - 2);
    }
    return c;
}

// With the tile-qubit search on, whole plans made with half and with all of
// the random restarts are compared by plan_cost: more restarts find sweeps
// that apply more gates, which is not always the cheaper plan (fewer sweeps
// carrying more blocks).  On states of at least 24 qubits the same two are
// made with lookaheads of three, four and five sweeps as well, each with a
// run weight of 0 and of 1: the search is greedy per sweep, and a wider set
// of plans gives the estimate more to choose from (on the 30-qubit depth-40
// circuit: 28 sweeps with 183-186 blocks against 195 with the two-sweep
// lookahead alone, and with a run weight of one 8 of the 28 tiles with
// qubits 0..5 against 3, 11970 against 11890 gates/s; on the 34-qubit
// depth-24 one a lookahead of three finds 12 sweeps with 96 blocks, which
// the estimate ranks behind 13 with 87, as measured).
void plan_tiles_variants(const std::vector<FlatOp> &flat, size_t k0, size_t e, int n, const TileParams &tp,
                         std::vector<std::vector<PlanStep>> &out)
{
    out.clear();
    if (!tp.search || tp.restarts < 2) {
        out.emplace_back();
        plan_tiles_once(flat, k0, e, n, tp, out.back());
        return;
    }
    std::vector<TileParams> vs;
    for (int rw = 0; rw <= (n >= 24 ? 1 : 0); ++rw)
        for (int la = 2; la <= (n >= 24 ? 5 : 2); ++la) {
            TileParams half = tp, all = tp;
            half.restarts = tp.restarts / 2;
            half.lookahead = all.lookahead = la;
            half.run_weight = all.run_weight = rw;
            vs.push_back(half);
            vs.push_back(all);
        }
    // the variants are independent: one thread each (plan_tiles_once only
    // reads the gate list); an exception in a thread (an allocation that
    // fails) is passed on to the caller after every thread has ended
    out.resize(vs.size());
    std::vector<std::exception_ptr> err(vs.size());
    std::vector<std::thread> th;
    for (size_t i = 1; i < vs.size(); ++i)
        th.emplace_back([&, i] {
            try {
                plan_tiles_once(flat, k0, e, n, vs[i], out[i]);
            } catch (...) {
                err[i] = std::current_exception();
            }
        });
    try {
        plan_tiles_once(flat, k0, e, n, vs[0], out[0]);
    } catch (...) {
        err[0] = std::current_exception();
    }
    for (std::thread &t : th) t.join();
    for (const std::exception_ptr &x : err)
        if (x) std::rethrow_exception(x);
}

void plan_tiles(const std::vector<FlatOp> &flat, size_t k0, size_t e, int n, const TileParams &tp,
                std::vector<PlanStep> &out)
{
    std::vector<std::vector<PlanStep>> v;
    plan_tiles_variants(flat, k0, e, n, tp, v);
    size_t bi = 0;
    for (size_t i = 1; i < v.size(); ++i)
        if (plan_cost(v[i]) < plan_cost(v[bi])) bi = i;
    out.insert(out.end(), std::make_move_iterator(v[bi].begin()), std::make_move_iterator(v[bi].end()));
}

}  // namespace qs
