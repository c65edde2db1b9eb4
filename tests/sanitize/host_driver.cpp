// Host-side planning code of libqs under AddressSanitizer and
// UndefinedBehaviorSanitizer: circuits built through the C ABI, then every
// planner that needs no device (tile planner with its qubit search, greedy
// block fusion, partial-amplitude cuts, script reader, single-amplitude
// graph and elimination order), including their error paths.  Built with
// the device halves of the HIP sources left out (host-only compilation), so
// no kernel is ever launched.  Exit status 0 = no finding.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qs.h"

namespace {

uint64_t g_rng = 0x243F6A8885A308D3ull;
uint64_t next()
{
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return g_rng;
}
double uni() { return double(next() >> 11) * 0x1.0p-53; }

// A random complex matrix of size d x d; diag = diagonal only, ident = identity.
std::vector<double> matrix(int d, int kind)
{
    std::vector<double> m(size_t(2) * d * d, 0.0);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const size_t k = size_t(r) * d + c;
            if (kind == 0) {
                m[2 * k] = uni() - 0.5;
                m[2 * k + 1] = uni() - 0.5;
            } else if (r == c) {
                const double a = kind == 1 ? 6.283185307179586 * uni() : 0.0;
                m[2 * k] = std::cos(a);
                m[2 * k + 1] = std::sin(a);
            }
        }
    return m;
}

// DAGGER groups open with probability 1/8 and close with 1/4 per gate; one
// circuit in ten is left with a group open (an error for every planner).
qs_circuit *random_circuit(int n, int count)
{
    qs_circuit *c = nullptr;
    if (qs_circuit_create(&c)) return nullptr;
    bool open = false;
    for (int i = 0; i < count; ++i) {
        const int nt = 1 + int(next() % 3), nc = int(next() % 3);
        if (nt + nc > n) continue;
        std::vector<int> q;
        while (int(q.size()) < nt + nc) {
            const int x = int(next() % uint64_t(n));
            bool dup = false;
            for (int y : q) dup = dup || y == x;
            if (!dup) q.push_back(x);
        }
        const int kind = int(next() % 4) == 0 ? 1 : (int(next() % 16) == 0 ? 2 : 0);
        const std::vector<double> m = matrix(1 << nt, kind);
        if (!open && int(next() % 8) == 0) {
            qs_circuit_begin_dagger(c);
            open = true;
        }
        qs_circuit_append_gate(c, q.data(), nt, q.data() + nt, nc, m.data());
        if (open && int(next() % 4) == 0) {
            qs_circuit_end_dagger(c);
            open = false;
        }
    }
    if (open && int(next() % 10) != 0) qs_circuit_end_dagger(c);
    return c;
}

int planned = 0;

int failures = 0;
void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (%s)\n", what, qs_last_error());
        ++failures;
    }
}

}  // namespace

int main()
{
    // planners on random circuits of every shape
    for (int trial = 0; trial < 30; ++trial) {
        const int n = 10 + int(next() % 25);
        qs_circuit *c = random_circuit(n, 20 + int(next() % 200));
        expect(c != nullptr, "circuit");
        if (!c) continue;
        int64_t sw = 0, bl = 0, lg = 0;
        for (int plan = 0; plan <= 1; ++plan)
            for (int dt = 1; dt <= 2; ++dt) {
                qs_run_opts o{};
                o.plan = plan;
                o.k_max = dt == 2 ? 2 + int(next() % 5) : 4 + int(next() % 2);
                o.tile_qubits = dt == 1 ? 10 + int(next() % 4) : 0;
                planned += qs_circuit_plan_info(c, n, qs_dtype(dt), &o, &sw, &bl, &lg) == QS_OK;
            }
        int cuts = 0;
        for (int k = 0; k < 4; ++k) qs_partial_cuts(c, n, next() & ((uint64_t(1) << n) - 1), &cuts);
        qs_single_info si{};
        if (n <= 16) qs_single_plan(c, n, int(next() % 4), &si);
        qs_circuit_destroy(c);
    }
    // grid circuits: depth-limited single-amplitude plans and tile plans with the search on
    for (int d = 4; d <= 10; d += 3) {
        qs_circuit *c = nullptr;
        qs_circuit_create(&c);
        const int R = 5, C = 6, n = R * C;
        const std::vector<double> h = matrix(2, 0), cz = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0,
                                                         0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 0};
        for (int l = 0; l < d; ++l) {
            for (int q = 0; q < n; ++q) qs_circuit_append_gate(c, &q, 1, nullptr, 0, h.data());
            for (int r = 0; r < R; ++r)
                for (int x = (l & 1); x + 1 < C; x += 2) {
                    const int t[2] = {r * C + x, r * C + x + 1};
                    qs_circuit_append_gate(c, t, 2, nullptr, 0, cz.data());
                }
        }
        int64_t sw = 0, bl = 0, lg = 0;
        qs_run_opts o{};
        o.plan = QS_PLAN_GREEDY;
        expect(qs_circuit_plan_info(c, n, QS_C64, &o, &sw, &bl, &lg) == QS_OK, "grid tile plan");
        qs_single_info si{};
        expect(qs_single_plan(c, n, 2, &si) == QS_OK, "grid single-amplitude plan");
        int cuts = 0;
        expect(qs_partial_cuts(c, n, (uint64_t(1) << 15) - 1, &cuts) == QS_OK, "grid cuts");
        qs_circuit_destroy(c);
    }
    // the script reader: valid scripts and malformed ones
    const char *scripts[] = {
        "QINIT 5\nH 1\nS 2\nX 2\nH 2\nCR 1,2,\"pi/2\"\nDAGGER\nH 0\nSWAP 0,2\nENDDAGGER\nPMEASURE 4,3,0\n",
        "QINIT 3\nCREG 2\nCONTROL 2\nRX 0, pi/3\nTOFFOLI 0,1,2\nENDCONTROL 2\nMEASURE 0,$1\n",
        "QINIT 4\nU4 0, 0.1, 0.2, 0.3, 0.4\nISWAP 1,2\nRY 3, -(pi+1)/4*2\nCZ 0,3\nPMEASURE 0\n",
        "QINIT 2\nH 5\n",
        "QINIT 2\nRX 0, (pi\n",
        "H 0\n",
        "QINIT 3\nDAGGER\nH 0\n",
        "QINIT 3\nCREG 1\nMEASURE 0,$4\n",
        "QINIT 2\nPMEASURE 0\nH 1\n",
        "QINIT 2\nFOO 1\n",
        "QINIT 2\nCNOT 0,0\n",
        "QINIT 2\nRZ 0, 1e999999\n",
        "",
        "QINIT 62\nH 61\n",
        "QINIT 3\nCONTROL 0\nCONTROL 1\nX 2\nENDCONTROL\nENDCONTROL\n",
    };
    for (const char *t : scripts) {
        qs_circuit *c = nullptr;
        qs_script_info info{};
        if (qs_script_parse(t, &c, &info) == QS_OK) qs_circuit_destroy(c);
    }
    // a long generated script
    std::string big = "QINIT 20\nCREG 20\n";
    for (int i = 0; i < 2000; ++i) {
        char line[128];
        std::snprintf(line, sizeof line, "RY %d, %.17g\nCNOT %d,%d\n", i % 20, uni() * 7, i % 20, (i + 7) % 20);
        big += line;
    }
    {
        qs_circuit *c = nullptr;
        qs_script_info info{};
        expect(qs_script_parse(big.c_str(), &c, &info) == QS_OK, "long script");
        if (c) qs_circuit_destroy(c);
    }
    expect(planned >= 70, "most random circuits planned");
    std::printf("sanitized host planning run: %d plans, %d failures\n", planned, failures);
    return failures ? 1 : 0;
}
