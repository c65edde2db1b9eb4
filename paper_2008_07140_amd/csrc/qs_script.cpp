// Input scripts in the instruction set of App. A-1: a parser that builds a
// circuit through the public circuit calls, and a runner that executes it on
// a new state and collects MEASURE outcomes and PMEASURE probabilities (the
// output of App. A-2; failures carry the line number, the counterpart of its
// error log).
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/qs.h"
#include "qs_plan.h"

namespace {

using cd = std::complex<double>;

struct ScriptError {
    qs_status st;
    std::string msg;
};

[[noreturn]] void raise(qs_status st, int line, const std::string &msg)
{
    throw ScriptError{st, "line " + std::to_string(line) + ": " + msg};
}

// ---------------------------------------------------------- angle values --

// number | pi | ( expr ) | -factor, combined with * / + -
struct Expr {
    const std::string &s;
    size_t i = 0;
    int line;
    void ws()
    {
        while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
    }
    double primary()
    {
        ws();
        if (i < s.size() && (s[i] == '-' || s[i] == '+')) {
            const bool neg = s[i++] == '-';
            const double v = primary();
            return neg ? -v : v;
        }
        if (i < s.size() && s[i] == '(') {
            ++i;
            const double v = sum();
            ws();
            if (i >= s.size() || s[i] != ')') raise(QS_E_INVAL, line, "missing ')' in \"" + s + "\"");
            ++i;
            return v;
        }
        if (s.compare(i, 2, "pi") == 0) {
            i += 2;
            return M_PI;
        }
        const char *b = s.c_str() + i;
        char *e = nullptr;
        const double v = std::strtod(b, &e);
        if (e == b) raise(QS_E_INVAL, line, "not a number: \"" + s + "\"");
        i += size_t(e - b);
        return v;
    }
    double product()
    {
        double v = primary();
        for (;;) {
            ws();
            if (i < s.size() && (s[i] == '*' || s[i] == '/')) {
                const bool mul = s[i++] == '*';
                const double r = primary();
                v = mul ? v * r : v / r;
            } else {
                return v;
            }
        }
    }
    double sum()
    {
        double v = product();
        for (;;) {
            ws();
            if (i < s.size() && (s[i] == '+' || s[i] == '-')) {
                const bool add = s[i++] == '+';
                const double r = product();
                v = add ? v + r : v - r;
            } else {
                return v;
            }
        }
    }
};

double angle(const std::string &tok, int line)
{
    std::string t;
    for (char ch : tok)
        if (ch != '"') t += char(std::tolower(static_cast<unsigned char>(ch)));
    Expr e{t, 0, line};
    const double v = e.sum();
    e.ws();
    if (e.i != t.size() || !std::isfinite(v)) raise(QS_E_INVAL, line, "bad angle \"" + tok + "\"");
    return v;
}

// -------------------------------------------------------------- gates --

// 2^k x 2^k matrix as the ABI takes it: row-major (re, im) pairs
std::vector<double> flat(const std::vector<cd> &u)
{
    std::vector<double> m;
    for (const cd &z : u) {
        m.push_back(z.real());
        m.push_back(z.imag());
    }
    return m;
}

// the one-qubit operators of App. A-1
std::vector<cd> one_qubit(const std::string &name, const std::vector<double> &p)
{
    const cd I(0, 1);
    const double r = std::sqrt(0.5);
    if (name == "H") return {r, r, r, -r};
    if (name == "X") return {0, 1, 1, 0};
    if (name == "Y") return {0, -I, I, 0};
    if (name == "Z") return {1, 0, 0, -1};
    if (name == "S") return {1, 0, 0, I};
    if (name == "T") return {1, 0, 0, std::polar(1.0, M_PI / 4)};
    const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
    if (name == "RX") return {c, -I * s, -I * s, c};
    if (name == "RY") return {c, -s, s, c};
    if (name == "RZ") return {std::polar(1.0, -p[0] / 2), 0, 0, std::polar(1.0, p[0] / 2)};
    // U4 (alpha, beta, gamma, delta)
    const double a = p[0], b = p[1], cg = std::cos(p[2] / 2), sg = std::sin(p[2] / 2), d = p[3];
    return {std::polar(cg, a - b / 2 - d / 2), -std::polar(sg, a - b / 2 + d / 2), std::polar(sg, a + b / 2 - d / 2),
            std::polar(cg, a + b / 2 + d / 2)};
}

struct Parsed {
    qs_circuit *c = nullptr;
    qs_script_info info{};
    std::vector<int> measure_reg;  // classical register of each MEASURE, in order
};

void check(qs_status st, int line)
{
    if (st != QS_OK) raise(st, line, qs_last_error());
}

void parse(const char *text, Parsed &P)
{
    std::vector<std::string> lines;
    {
        std::string cur;
        for (const char *p = text; *p; ++p) {
            if (*p == '\n') {
                lines.push_back(cur);
                cur.clear();
            } else {
                cur += *p;
            }
        }
        lines.push_back(cur);
    }
    int n = -1;
    bool pm_seen = false;
    std::vector<int> groups;  // open groups: -1 = DAGGER, q = CONTROL q
    std::vector<int> opened;  // their lines
    check(qs_circuit_create(&P.c), 0);
    for (size_t li = 0; li < lines.size(); ++li) {
        const int line = int(li) + 1;
        std::string s = lines[li].substr(0, lines[li].find('#'));
        while (!s.empty() && std::isspace(static_cast<unsigned char>(s.back()))) s.pop_back();
        size_t b = 0;
        while (b < s.size() && std::isspace(static_cast<unsigned char>(s[b]))) ++b;
        s = s.substr(b);
        if (s.empty() || s[0] == '%') continue;
        size_t sp = 0;
        while (sp < s.size() && !std::isspace(static_cast<unsigned char>(s[sp]))) ++sp;
        std::string name = s.substr(0, sp);
        for (char &ch : name) ch = char(std::toupper(static_cast<unsigned char>(ch)));
        // arguments: split on commas, quotes removed
        std::vector<std::string> args;
        {
            std::string rest = s.substr(sp), cur;
            bool any = false;
            for (char ch : rest) {
                if (ch == ',') {
                    args.push_back(cur);
                    cur.clear();
                    any = true;
                } else if (ch != '"') {
                    cur += ch;
                    if (!std::isspace(static_cast<unsigned char>(ch))) any = true;
                }
            }
            if (any) args.push_back(cur);
            for (auto &a : args) {
                size_t x = 0, y = a.size();
                while (x < y && std::isspace(static_cast<unsigned char>(a[x]))) ++x;
                while (y > x && std::isspace(static_cast<unsigned char>(a[y - 1]))) --y;
                a = a.substr(x, y - x);
            }
        }
        auto need = [&](size_t k) {
            if (args.size() != k)
                raise(QS_E_INVAL, line, name + " takes " + std::to_string(k) + " arguments, got " +
                                            std::to_string(args.size()));
        };
        auto integer = [&](const std::string &a, bool reg = false) {
            std::string t = a;
            if (reg) {
                if (t.empty() || t[0] != '$') raise(QS_E_INVAL, line, "register \"" + a + "\" must start with $");
                t = t.substr(1);
            }
            char *e = nullptr;
            const long v = std::strtol(t.c_str(), &e, 10);
            if (t.empty() || *e) raise(QS_E_INVAL, line, "not an integer: \"" + a + "\"");
            return v;
        };
        auto qubit = [&](const std::string &a) {
            const long q = integer(a);
            if (q < 0 || q >= n) raise(QS_E_RANGE, line, "qubit " + a + " not in [0, " + std::to_string(n) + ")");
            return int(q);
        };
        if (pm_seen) raise(QS_E_INVAL, line, "PMEASURE must be the last instruction");
        if (name == "QINIT") {
            need(1);
            if (n >= 0) raise(QS_E_INVAL, line, "second QINIT");
            const long v = integer(args[0]);
            if (v < 1 || v > QS_MAX_QUBITS)
                raise(QS_E_INVAL, line, "QINIT " + args[0] + " not in [1, " + std::to_string(QS_MAX_QUBITS) + "]");
            n = int(v);
            P.info.n = n;
            continue;
        }
        if (n < 0) raise(QS_E_INVAL, line, "QINIT must come first");
        if (name == "CREG") {
            need(1);
            const long v = integer(args[0]);
            if (v < 0 || v > (1 << 20)) raise(QS_E_INVAL, line, "CREG " + args[0] + " out of range");
            P.info.creg = int(v);
        } else if (name == "H" || name == "X" || name == "Y" || name == "Z" || name == "S" || name == "T") {
            need(1);
            const int q = qubit(args[0]);
            check(qs_circuit_append_gate(P.c, &q, 1, nullptr, 0, flat(one_qubit(name, {})).data()), line);
        } else if (name == "RX" || name == "RY" || name == "RZ") {
            need(2);
            const int q = qubit(args[0]);
            check(qs_circuit_append_gate(P.c, &q, 1, nullptr, 0, flat(one_qubit(name, {angle(args[1], line)})).data()),
                  line);
        } else if (name == "U4") {
            need(5);
            const int q = qubit(args[0]);
            std::vector<double> p;
            for (int k = 1; k < 5; ++k) p.push_back(angle(args[k], line));
            check(qs_circuit_append_gate(P.c, &q, 1, nullptr, 0, flat(one_qubit("U4", p)).data()), line);
        } else if (name == "CNOT" || name == "CZ" || name == "CR") {
            need(name == "CR" ? 3 : 2);
            const int ctl = qubit(args[0]), tgt = qubit(args[1]);
            std::vector<cd> u = name == "CNOT" ? one_qubit("X", {}) : one_qubit("Z", {});
            if (name == "CR") u = {1, 0, 0, std::polar(1.0, angle(args[2], line))};
            check(qs_circuit_append_gate(P.c, &tgt, 1, &ctl, 1, flat(u).data()), line);
        } else if (name == "SWAP" || name == "ISWAP") {
            need(2);
            const int t[2] = {qubit(args[0]), qubit(args[1])};
            const cd x = name == "SWAP" ? cd(1) : cd(0, -1);
            const std::vector<cd> u = {1, 0, 0, 0, 0, 0, x, 0, 0, x, 0, 0, 0, 0, 0, 1};
            check(qs_circuit_append_gate(P.c, t, 2, nullptr, 0, flat(u).data()), line);
        } else if (name == "TOFFOLI") {
            need(3);
            const int ctl[2] = {qubit(args[0]), qubit(args[1])}, tgt = qubit(args[2]);
            check(qs_circuit_append_gate(P.c, &tgt, 1, ctl, 2, flat(one_qubit("X", {})).data()), line);
        } else if (name == "DAGGER") {
            need(0);
            groups.push_back(-1);
            opened.push_back(line);
            check(qs_circuit_begin_dagger(P.c), line);
        } else if (name == "ENDDAGGER") {
            need(0);
            if (groups.empty() || groups.back() != -1) raise(QS_E_INVAL, line, "ENDDAGGER without DAGGER");
            groups.pop_back();
            opened.pop_back();
            check(qs_circuit_end_dagger(P.c), line);
        } else if (name == "CONTROL") {
            need(1);
            const int q = qubit(args[0]);
            groups.push_back(q);
            opened.push_back(line);
            check(qs_circuit_begin_control(P.c, q), line);
        } else if (name == "ENDCONTROL") {
            if (args.size() > 1) need(1);
            if (groups.empty() || groups.back() < 0) raise(QS_E_INVAL, line, "ENDCONTROL without CONTROL");
            if (args.size() == 1 && qubit(args[0]) != groups.back())
                raise(QS_E_INVAL, line, "ENDCONTROL " + args[0] + " closes CONTROL " + std::to_string(groups.back()));
            groups.pop_back();
            opened.pop_back();
            check(qs_circuit_end_control(P.c), line);
        } else if (name == "MEASURE") {
            need(2);
            const int q = qubit(args[0]);
            const long r = integer(args[1], true);
            if (r < 0 || r >= P.info.creg)
                raise(QS_E_RANGE, line, "register " + args[1] + " not among the " + std::to_string(P.info.creg) +
                                            " of CREG");
            if (!groups.empty()) raise(QS_E_UNSUPPORTED, line, "MEASURE inside a DAGGER or CONTROL group");
            const std::vector<cd> id = {1, 0, 0, 1}, p0 = {1, 0, 0, 0}, p1 = {0, 0, 0, 1};
            check(qs_circuit_append_gate(P.c, &q, 1, nullptr, 0, flat(id).data()), line);
            std::vector<double> k = flat(p0), k1 = flat(p1);
            k.insert(k.end(), k1.begin(), k1.end());
            check(qs_circuit_append_noise(P.c, &q, 1, k.data(), 2), line);
            P.measure_reg.push_back(int(r));
            P.info.measures++;
        } else if (name == "PMEASURE") {
            if (args.empty() || int(args.size()) > n)
                raise(QS_E_INVAL, line, "PMEASURE takes 1 to " + std::to_string(n) + " qubits");
            uint64_t seen = 0;
            for (size_t k = 0; k < args.size(); ++k) {
                const int q = qubit(args[k]);
                if ((seen >> q) & 1) raise(QS_E_RANGE, line, "qubit " + args[k] + " listed twice");
                seen |= uint64_t(1) << q;
                P.info.pmeasure[k] = q;
            }
            if (!groups.empty()) raise(QS_E_INVAL, line, "PMEASURE inside a group");
            P.info.pmeasure_n = int(args.size());
            pm_seen = true;
        } else {
            raise(QS_E_INVAL, line, "unknown instruction " + name);
        }
    }
    if (n < 0) raise(QS_E_INVAL, 1, "no QINIT");
    if (!groups.empty())
        raise(QS_E_INVAL, opened.back(), groups.back() < 0 ? "DAGGER without ENDDAGGER" : "CONTROL without ENDCONTROL");
}

}  // namespace

extern "C" {

qs_status qs_script_parse(const char *text, qs_circuit **circuit, qs_script_info *info)
{
    if (!text || !circuit) return qs::set_error(QS_E_INVAL, "text or circuit is NULL");
    *circuit = nullptr;
    Parsed P;
    try {
        parse(text, P);
    } catch (const ScriptError &e) {
        qs_circuit_destroy(P.c);
        return qs::set_error(e.st, e.msg.c_str());
    } catch (const std::bad_alloc &) {
        qs_circuit_destroy(P.c);
        return qs::set_error(QS_E_NOMEM, "host allocation failed while reading the script");
    } catch (const std::exception &e) {  // nothing may unwind through the C ABI
        qs_circuit_destroy(P.c);
        return qs::set_error(QS_E_INVAL, e.what());
    }
    *circuit = P.c;
    if (info) *info = P.info;
    return QS_OK;
}

qs_status qs_script_run(const char *text, qs_dtype dt, uint64_t seed, int plan, int *creg, int creg_len,
                        double *probs, size_t probs_len, qs_script_info *info)
{
    if (!text) return qs::set_error(QS_E_INVAL, "text is NULL");
    if (plan < QS_PLAN_UNFUSED || plan >= QS_PLAN_AUTOTUNE) return qs::set_error(QS_E_INVAL, "plan not accepted");
    Parsed P;
    try {
        parse(text, P);
    } catch (const ScriptError &e) {
        qs_circuit_destroy(P.c);
        return qs::set_error(e.st, e.msg.c_str());
    } catch (const std::bad_alloc &) {
        qs_circuit_destroy(P.c);
        return qs::set_error(QS_E_NOMEM, "host allocation failed while reading the script");
    } catch (const std::exception &e) {  // nothing may unwind through the C ABI
        qs_circuit_destroy(P.c);
        return qs::set_error(QS_E_INVAL, e.what());
    }
    const qs_script_info &I = P.info;
    qs_status st = QS_OK;
    if (I.creg > 0 && (!creg || creg_len < I.creg))
        st = qs::set_error(QS_E_INVAL, "creg output shorter than CREG");
    else if (I.pmeasure_n > 0 && (!probs || probs_len < (size_t(1) << I.pmeasure_n)))
        st = qs::set_error(QS_E_INVAL, "probability output shorter than 2^(PMEASURE qubits)");
    qs_state *s = nullptr;
    if (st == QS_OK) st = qs_create(I.n, dt, &s);
    if (st == QS_OK) {
        std::vector<int64_t> chosen(P.measure_reg.size() + 1, 0);
        qs_run_opts o{};
        o.plan = I.measures ? QS_PLAN_UNFUSED : plan;
        o.seed = seed;
        o.chosen = chosen.data();
        o.chosen_len = int64_t(P.measure_reg.size());
        st = qs_run_circuit(s, P.c, &o);
        if (st == QS_OK && I.pmeasure_n > 0) st = qs_probabilities(s, I.pmeasure, I.pmeasure_n, probs);
        if (st == QS_OK) st = qs_synchronize(s);
        if (st == QS_OK && creg) {
            for (int j = 0; j < I.creg; ++j) creg[j] = 0;
            for (size_t k = 0; k < P.measure_reg.size(); ++k) creg[P.measure_reg[k]] = int(chosen[k]);
        }
    }
    if (s) qs_destroy(s);
    qs_circuit_destroy(P.c);
    if (st == QS_OK && info) *info = I;
    return st;
}

}  // extern "C"
