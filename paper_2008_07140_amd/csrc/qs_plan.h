// Circuit representation, group expansion, gate canonicalisation and the
// fusion planner (host side).
#pragma once

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

qs_status run_trajectories(const qs_circuit *const *circs, const int *widths, int count, qs_dtype dt,
                           uint64_t seed, double *z_out, double *seconds);

qs_status set_error(qs_status st, const char *msg);
qs_status run_on_state(qs_state *s, const qs_circuit *c, const qs_run_opts *o);

}  // namespace qs
