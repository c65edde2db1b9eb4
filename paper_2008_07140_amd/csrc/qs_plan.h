// Circuit representation, group expansion, gate canonicalisation and the
// fusion planner (host side).
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "qs_internal.h"

namespace qs {

// One entry of a circuit as appended through the ABI.
struct Op {
    enum Kind { GATE, NOISE, BEGIN_DAGGER, END_DAGGER, BEGIN_CONTROL, END_CONTROL };
    Kind kind = GATE;
    std::vector<int> targets, controls;
    std::vector<double> m;  // gate matrix, or nk Kraus matrices one after another
    int nk = 0;
    int qubit = -1;         // BEGIN_CONTROL
};

// A gate or noise site after DAGGER / CONTROL expansion.
struct FlatOp {
    enum Kind { GATE, NOISE };
    Kind kind = GATE;
    std::vector<int> targets, controls;
    std::vector<double> m;
    int nk = 0;
};

// A gate in the form the kernels take.
struct CanonGate {
    enum Kind { IDENTITY, PHASE, DENSE };
    Kind kind = IDENTITY;
    std::vector<int> targets;   // targets[0] = most significant bit of the matrix index
    std::vector<int> controls;
    std::vector<double> m;      // DENSE: 2^nt x 2^nt; PHASE: 2^nt diagonal factors ((re, im) pairs)
};

// Expand DAGGER / CONTROL groups (App. A-1).  Returns 0, 1 for malformed
// groups, 2 for a noise site inside a group; err describes the problem.
int expand(const std::vector<Op> &ops, std::vector<FlatOp> &out, std::string &err);

// Bring a gate to canonical form: every target on which the matrix acts as
// the identity unless that bit is 1 becomes a control; diagonal matrices
// become PHASE; the identity becomes IDENTITY.
CanonGate canonicalize(const int *t, int nt, const int *c, int nc, const double *m);

bool is_identity(const std::vector<double> &m, int nt);

// Fuse flat gates [k, e) into dense blocks of at most kmax qubits.
void greedy_fuse(const std::vector<FlatOp> &flat, size_t k, size_t e, int kmax,
                 std::vector<CanonGate> &plan);

int default_kmax(int n, qs_dtype dt);
int default_tile_qubits(int n);

qs_status set_error(qs_status st, const char *msg);
qs_status run_on_state(qs_state *s, const qs_circuit *c, const qs_run_opts *o);
// The ops of a circuit as appended (groups not yet expanded).
const std::vector<Op> &circuit_ops(const qs_circuit *c);
// Plans of other modes kept with a circuit, by key; dropped when the
// circuit changes (thread-safe).
std::shared_ptr<const void> circuit_cache_get(const qs_circuit *c, uint64_t key);
void circuit_cache_put(const qs_circuit *c, uint64_t key, std::shared_ptr<const void> v);
// The process-wide qs_set_memory_limit bound (0 = none).
size_t memory_limit();

}  // namespace qs

namespace qs {

// ---------------------------------------------------------------- tiles --
// A tile sweep keeps 2^m amplitudes of the qubit set Q (ascending, always
// starting with the L lowest qubits) in LDS and applies a list of ops to
// every tile; the other n - m bits index the tiles.

constexpr int kMaxOuter = 5;  // outer selector bits of one tile op

struct TileOp {
    enum Kind { DENSE, PHASE };
    Kind kind = DENSE;
    // `qubits` lie in Q (qubits[0] = most significant bit of a matrix index),
    // `outer` outside Q (at most kMaxOuter, outer[0] most significant); the outer
    // bits are constant over a tile and select one of 2^|outer| operators.
    // DENSE: m holds the distinct matrices (2^k x 2^k complex) one after
    // another and pmap[p] is the matrix of outer pattern p; `skip` bit p is
    // set when that matrix is the identity.
    // PHASE: m is the diagonal table, entry (outer pattern << k) | (qubit
    // pattern).
    std::vector<int> qubits;
    std::vector<int> outer;
    std::vector<double> m;
    std::vector<uint8_t> pmap;
    uint32_t skip = 0;
};

struct Sweep {
    std::vector<int> Q;
    std::vector<TileOp> ops;
    int gates = 0;  // logical gates applied in this sweep
};

struct TileParams {
    int m = 12;     // tile qubits
    int L = 4;      // lowest qubits always in the tile
    int kmax = 4;   // widest dense block (4 or 5)
    int max_outer = kMaxOuter;  // outer selector bits per op (0..kMaxOuter)
    bool search = true;  // improve each sweep's tile qubits by local search
    int restarts = 32;   // extra random starting sets for that search
    int lookahead = 2;   // sweeps scored per candidate tile set
    int run_weight = 0;  // gates a tile set may give up per extra low qubit beyond the four (at most two)
};

// One step of a tiled plan: a tile sweep, or a gate that does not fit a tile
// (more qubits than kmax) applied by the per-gate kernels.
struct PlanStep {
    bool sweep = true;
    Sweep sw;
    CanonGate gate;
};

// Plan the gates flat[k, e) as tile sweeps (appended to out): of the whole
// plans made with half and with all of tp.restarts (and, on states of at
// least 24 qubits, the same two with lookaheads of three to five sweeps,
// each also with a run weight of one), the one with the lower fixed cost
// estimate.
void plan_tiles(const std::vector<FlatOp> &flat, size_t k, size_t e, int n, const TileParams &tp,
                std::vector<PlanStep> &out);
// The candidate whole plans plan_tiles chooses between (one when the search
// is off), for a cost model to choose instead.
void plan_tiles_variants(const std::vector<FlatOp> &flat, size_t k, size_t e, int n, const TileParams &tp,
                         std::vector<std::vector<PlanStep>> &out);
// The fixed estimate plan_tiles ranks them by (memory passes, shorter for
// tiles whose qubits 0..4 or 0..5 are contiguous, plus 0.15 per dense block
// beyond two per sweep).
double plan_cost(const std::vector<PlanStep> &steps);

}  // namespace qs
