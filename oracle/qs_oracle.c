/*
 * qs_oracle.c -- FP64 CPU oracle for the full-amplitude state-vector method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library: both sides only read the same seeded circuit description.
 *
 * Paper: Wang et al., "A quantum circuit simulator and its applications on
 * Sunway TaihuLight supercomputer" (arXiv:2008.07140).
 *
 *  - State: 2^n complex amplitudes, qubit k is bit k of the index (Sec. 2.2,
 *    Eq. 1).  Initial state |0...0> (App. A-1, QINIT).
 *  - Gate update: the pair update of Eq. 2 for one target and its controlled
 *    form Eq. 3, generalised in the obvious way to a dense 2^nt x 2^nt matrix
 *    on nt target qubits (the group gathered by fixing every other bit).  Row
 *    index of a multi-qubit matrix: targets[0] is its most significant bit,
 *    as the CNOT/TOFFOLI matrices of App. A-1 print them (first listed qubit
 *    is the control = high bit of the row index).
 *  - Named gates: the matrices printed in App. A-1.
 *  - DAGGER / CONTROL groups: App. A-1 (nestable).
 *  - Noisy gate: the three steps of Sec. 2.4 taken literally (every Kraus
 *    operator applied to a full copy of the post-gate state, probabilities
 *    from the copies, branch picked by a uniform number against the running
 *    sum, the product K_b*U applied to the state, then the state normalised).
 *  - PMEASURE: probabilities of the listed qubits, first listed = most
 *    significant bit of the output index (App. A-1 and the worked example of
 *    App. A-2).
 *  - Density matrix (n <= 10): rho <- U rho U^dagger, rho <- sum_b K_b rho
 *    K_b^dagger; the ensemble the trajectories of Sec. 2.4 sample from.
 *  - Philox4x32-10 counter-based generator (Salmon et al., SC'11), written
 *    from its published definition, for the uniform numbers of Sec. 2.4 step 2.
 *  - A small fully connected network (F -> 64 -> 64 -> 1, ReLU) in FP64 with
 *    its exact backward pass: the reference for the cost-model kernels.
 *
 * Everything is FP64 (double complex).  No blocking, fusion or reordering.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_MAX_T 8 /* largest dense gate the oracle accepts: 2^8 x 2^8 */

/* Threads the OpenMP loops of the oracle use. */
int or_num_threads(void) { return omp_get_max_threads(); }

/* Set that number (k >= 1), for timing the oracle on fewer host threads. */
void or_set_threads(int k)
{
    if (k >= 1) omp_set_num_threads(k);
}

/* ------------------------------------------------------------------ */
/* State                                                               */
/* ------------------------------------------------------------------ */

/* |0...0>: alpha_0 = 1, all others 0 (App. A-1 QINIT). */
void or_init(cplx *psi, int n)
{
    uint64_t dim = (uint64_t)1 << n;
    memset(psi, 0, dim * sizeof(cplx));
    psi[0] = 1.0;
}

double or_norm2(const cplx *psi, int n)
{
    uint64_t dim = (uint64_t)1 << n;
    double s = 0.0;
    for (uint64_t i = 0; i < dim; ++i) {
        double re = creal(psi[i]), im = cimag(psi[i]);
        s += re * re + im * im;
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Gate application: Eq. 2 (one target), Eq. 3 (controls), generalised */
/* to nt targets.                                                      */
/* ------------------------------------------------------------------ */

static int check_qubit_list(int n, const int *t, int nt, const int *c, int nc, int max_nt)
{
    uint64_t seen = 0;
    if (nt < 0 || nt > max_nt || nc < 0 || nt + nc > n) return -1;
    for (int a = 0; a < nt + nc; ++a) {
        int q = a < nt ? t[a] : c[a - nt];
        if (q < 0 || q >= n) return -1;
        if (seen & ((uint64_t)1 << q)) return -1;
        seen |= (uint64_t)1 << q;
    }
    return 0;
}

static int check_qubits(int n, const int *t, int nt, const int *c, int nc)
{
    return check_qubit_list(n, t, nt, c, nc, OR_MAX_T);
}

/*
 * Apply the 2^nt x 2^nt row-major matrix m to the targets, conditioned on
 * every control qubit being |1>.  For every index i whose target bits are all
 * 0 and whose control bits are all 1, the 2^nt amplitudes obtained by setting
 * the target bits to every pattern x are gathered (bit b of the pattern, from
 * the top, goes to targets[b]), multiplied by m, and written back.
 * Returns 0, or -1 on invalid qubits.
 */
int or_apply(cplx *psi, int n, const int *targets, int nt,
             const int *controls, int nc, const cplx *m)
{
    if (check_qubits(n, targets, nt, controls, nc)) return -1;
    uint64_t dim = (uint64_t)1 << n;
    uint64_t tmask = 0, cmask = 0;
    for (int b = 0; b < nt; ++b) tmask |= (uint64_t)1 << targets[b];
    for (int b = 0; b < nc; ++b) cmask |= (uint64_t)1 << controls[b];
    int gsz = 1 << nt;
    uint64_t off[1 << OR_MAX_T];
    for (int x = 0; x < gsz; ++x) {
        uint64_t o = 0;
        for (int b = 0; b < nt; ++b)
            if ((x >> (nt - 1 - b)) & 1) o |= (uint64_t)1 << targets[b];
        off[x] = o;
    }
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & tmask) != 0 || (i & cmask) != cmask) continue;
        cplx v[1 << OR_MAX_T], w[1 << OR_MAX_T];
        for (int x = 0; x < gsz; ++x) v[x] = psi[i | off[x]];
        for (int r = 0; r < gsz; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < gsz; ++c) acc += m[(size_t)r * gsz + c] * v[c];
            w[r] = acc;
        }
        for (int x = 0; x < gsz; ++x) psi[i | off[x]] = w[x];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* PMEASURE (App. A-1): marginal probabilities of the listed qubits.  */
/* Output index bit (nq-1-b) is the value of qubits[b].               */
/* ------------------------------------------------------------------ */
int or_probabilities(const cplx *psi, int n, const int *qubits, int nq, double *out)
{
    if (check_qubit_list(n, qubits, nq, NULL, 0, n)) return -1;
    uint64_t dim = (uint64_t)1 << n;
    memset(out, 0, ((size_t)1 << nq) * sizeof(double));
    for (uint64_t i = 0; i < dim; ++i) {
        uint64_t x = 0;
        for (int b = 0; b < nq; ++b) x = (x << 1) | ((i >> qubits[b]) & 1);
        double re = creal(psi[i]), im = cimag(psi[i]);
        out[x] += re * re + im * im;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Named gates of App. A-1.  Writes the row-major matrix into m and    */
/* returns the number of qubits it acts on (first listed = MSB), or -1. */
/* params: RX/RY/RZ/CR use params[0] = theta; U4 with kind "U4E" takes  */
/* four complex elements as 8 doubles (re,im)*4, kind "U4" takes the   */
/* angles alpha, beta, gamma, delta.                                   */
/* ------------------------------------------------------------------ */
int or_named_gate(const char *name, const double *params, cplx *m)
{
    const double s2 = sqrt(0.5);
    memset(m, 0, 64 * sizeof(cplx));
    if (!strcmp(name, "H")) {
        m[0] = s2; m[1] = s2; m[2] = s2; m[3] = -s2; return 1;
    }
    if (!strcmp(name, "X")) { m[1] = 1; m[2] = 1; return 1; }
    if (!strcmp(name, "Y")) { m[1] = -I; m[2] = I; return 1; }
    if (!strcmp(name, "Z")) { m[0] = 1; m[3] = -1; return 1; }
    if (!strcmp(name, "S")) { m[0] = 1; m[3] = I; return 1; }
    if (!strcmp(name, "T")) { m[0] = 1; m[3] = cexp(I * M_PI / 4); return 1; }
    if (!strcmp(name, "RX")) {
        double c = cos(params[0] / 2), s = sin(params[0] / 2);
        m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; return 1;
    }
    if (!strcmp(name, "RY")) {
        double c = cos(params[0] / 2), s = sin(params[0] / 2);
        m[0] = c; m[1] = -s; m[2] = s; m[3] = c; return 1;
    }
    if (!strcmp(name, "RZ")) {
        m[0] = cexp(-I * params[0] / 2); m[3] = cexp(I * params[0] / 2); return 1;
    }
    if (!strcmp(name, "U4E")) {
        for (int k = 0; k < 4; ++k) m[k] = params[2 * k] + I * params[2 * k + 1];
        return 1;
    }
    if (!strcmp(name, "U4")) {
        double al = params[0], be = params[1], ga = params[2], de = params[3];
        double c = cos(ga / 2), s = sin(ga / 2);
        m[0] = cexp(I * (al - be / 2 - de / 2)) * c;
        m[1] = -cexp(I * (al - be / 2 + de / 2)) * s;
        m[2] = cexp(I * (al + be / 2 - de / 2)) * s;
        m[3] = cexp(I * (al + be / 2 + de / 2)) * c;
        return 1;
    }
    if (!strcmp(name, "CNOT")) {
        m[0] = 1; m[5] = 1; m[11] = 1; m[14] = 1; return 2;
    }
    if (!strcmp(name, "CZ")) {
        m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1; return 2;
    }
    if (!strcmp(name, "CR")) {
        m[0] = 1; m[5] = 1; m[10] = 1; m[15] = cexp(I * params[0]); return 2;
    }
    if (!strcmp(name, "SWAP")) {
        m[0] = 1; m[6] = 1; m[9] = 1; m[15] = 1; return 2;
    }
    if (!strcmp(name, "ISWAP")) {
        m[0] = 1; m[6] = -I; m[9] = -I; m[15] = 1; return 2;
    }
    if (!strcmp(name, "TOFFOLI")) {
        for (int k = 0; k < 6; ++k) m[k * 8 + k] = 1;
        m[6 * 8 + 7] = 1; m[7 * 8 + 6] = 1; return 3;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                 */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * The uniform number for noise site `site` of trajectory `traj` under `seed`:
 * counter = (site lo, site hi, traj lo, traj hi), key = (seed lo, seed hi);
 * the first two output words form a 64-bit integer x (word 1 high) and
 * u = (x >> 11) * 2^-53, so u lies in [0, 1).
 */
double or_uniform(uint64_t seed, uint64_t traj, uint64_t site)
{
    uint32_t ctr[4] = {(uint32_t)site, (uint32_t)(site >> 32),
                       (uint32_t)traj, (uint32_t)(traj >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    uint64_t x = ((uint64_t)o[1] << 32) | o[0];
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* Noisy gate, Sec. 2.4, taken step by step.                           */
/* ------------------------------------------------------------------ */

static void matmul(const cplx *a, const cplx *b, cplx *c, int d)
{
    for (int r = 0; r < d; ++r)
        for (int k = 0; k < d; ++k) {
            cplx acc = 0.0;
            for (int j = 0; j < d; ++j) acc += a[r * d + j] * b[j * d + k];
            c[r * d + k] = acc;
        }
}

/*
 * psi: state; m: the gate U on `targets` (2^nt x 2^nt); kraus: nk operators
 * of the same size stored one after another.  u in [0,1).
 * Step 1: apply U to a copy of the state, then every K_b to its own copy of
 *         that, and take p_b = ||K_b U psi||^2.
 * Step 2: b = first index with u < p_0 + ... + p_b (if rounding leaves u
 *         beyond the total, the last b with p_b > 0).
 * Step 3: psi <- (K_b U) psi, then psi <- psi / ||psi||.
 * Returns 0, -1 on invalid qubits, -2 if every p_b is 0.
 */
int or_apply_noisy(cplx *psi, int n, const int *targets, int nt, const cplx *m,
                   const cplx *kraus, int nk, double u, int *chosen, double *p_chosen,
                   double *probs_out)
{
    if (check_qubits(n, targets, nt, NULL, 0)) return -1;
    uint64_t dim = (uint64_t)1 << n;
    int d = 1 << nt;
    cplx *post = malloc(dim * sizeof(cplx));
    cplx *copy = malloc(dim * sizeof(cplx));
    double *p = malloc((size_t)nk * sizeof(double));
    memcpy(post, psi, dim * sizeof(cplx));
    or_apply(post, n, targets, nt, NULL, 0, m);
    for (int b = 0; b < nk; ++b) {
        memcpy(copy, post, dim * sizeof(cplx));
        or_apply(copy, n, targets, nt, NULL, 0, kraus + (size_t)b * d * d);
        p[b] = or_norm2(copy, n);
        if (probs_out) probs_out[b] = p[b];
    }
    int pick = -1;
    double run = 0.0;
    for (int b = 0; b < nk; ++b) {
        run += p[b];
        if (u < run) { pick = b; break; }
    }
    if (pick < 0)
        for (int b = nk - 1; b >= 0; --b)
            if (p[b] > 0) { pick = b; break; }
    if (pick < 0) { free(post); free(copy); free(p); return -2; }
    cplx *noisy = malloc((size_t)d * d * sizeof(cplx));
    matmul(kraus + (size_t)pick * d * d, m, noisy, d);
    or_apply(psi, n, targets, nt, NULL, 0, noisy);
    double nrm = sqrt(or_norm2(psi, n));
    for (uint64_t i = 0; i < dim; ++i) psi[i] /= nrm;
    *chosen = pick;
    *p_chosen = p[pick];
    free(noisy); free(post); free(copy); free(p);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Density matrix, n <= 10.  rho is 2^n x 2^n row-major.               */
/* ------------------------------------------------------------------ */

/* rho <- G rho G^dagger, G = the gate (targets, controls, m) on n qubits. */
int or_dm_apply(cplx *rho, int n, const int *targets, int nt,
                const int *controls, int nc, const cplx *m)
{
    if (check_qubits(n, targets, nt, controls, nc)) return -1;
    uint64_t dim = (uint64_t)1 << n;
    int d = 1 << nt;
    cplx *conjm = malloc((size_t)d * d * sizeof(cplx));
    for (int k = 0; k < d * d; ++k) conjm[k] = conj(m[k]);
    cplx *vec = malloc(dim * sizeof(cplx));
    /* columns: rho <- G rho */
    for (uint64_t c = 0; c < dim; ++c) {
        for (uint64_t r = 0; r < dim; ++r) vec[r] = rho[r * dim + c];
        or_apply(vec, n, targets, nt, controls, nc, m);
        for (uint64_t r = 0; r < dim; ++r) rho[r * dim + c] = vec[r];
    }
    /* rows: (rho G^dagger)[r, :] = conj(G) applied to row r */
    for (uint64_t r = 0; r < dim; ++r) {
        for (uint64_t c = 0; c < dim; ++c) vec[c] = rho[r * dim + c];
        or_apply(vec, n, targets, nt, controls, nc, conjm);
        for (uint64_t c = 0; c < dim; ++c) rho[r * dim + c] = vec[c];
    }
    free(vec); free(conjm);
    return 0;
}

/* rho <- sum_b K_b rho K_b^dagger. */
int or_dm_channel(cplx *rho, int n, const int *targets, int nt, const cplx *kraus, int nk)
{
    if (check_qubits(n, targets, nt, NULL, 0)) return -1;
    uint64_t dim = (uint64_t)1 << n;
    int d = 1 << nt;
    cplx *acc = calloc(dim * dim, sizeof(cplx));
    cplx *tmp = malloc(dim * dim * sizeof(cplx));
    for (int b = 0; b < nk; ++b) {
        memcpy(tmp, rho, dim * dim * sizeof(cplx));
        or_dm_apply(tmp, n, targets, nt, NULL, 0, kraus + (size_t)b * d * d);
        for (uint64_t k = 0; k < dim * dim; ++k) acc[k] += tmp[k];
    }
    memcpy(rho, acc, dim * dim * sizeof(cplx));
    free(acc); free(tmp);
    return 0;
}

/* <Z_q> = sum_x rho_xx (1 - 2 x_q) for every qubit q. */
void or_dm_expect_z(const cplx *rho, int n, double *out)
{
    uint64_t dim = (uint64_t)1 << n;
    for (int q = 0; q < n; ++q) {
        double s = 0.0;
        for (uint64_t x = 0; x < dim; ++x)
            s += creal(rho[x * dim + x]) * (((x >> q) & 1) ? -1.0 : 1.0);
        out[q] = s;
    }
}

/* <Z_q> of a pure state for every qubit q. */
void or_expect_z(const cplx *psi, int n, double *out)
{
    uint64_t dim = (uint64_t)1 << n;
    for (int q = 0; q < n; ++q) out[q] = 0.0;
    for (uint64_t x = 0; x < dim; ++x) {
        double re = creal(psi[x]), im = cimag(psi[x]);
        double pr = re * re + im * im;
        for (int q = 0; q < n; ++q) out[q] += ((x >> q) & 1) ? -pr : pr;
    }
}

/* ------------------------------------------------------------------ */
/* Circuits with DAGGER / CONTROL groups (App. A-1) and noise sites.  */
/*                                                                     */
/* An op list is given as parallel arrays: kind[k] is                  */
/*   0 gate   (nt[k] targets, nc[k] controls, matrix at mat_off[k])    */
/*   1 noise  (nt[k] targets, nk[k] Kraus matrices at mat_off[k]);     */
/*            the channel acts after the preceding gate, so the pair   */
/*            (gate, noise) is the noisy gate K_b*U of Sec. 2.4        */
/*   2 DAGGER, 3 ENDDAGGER, 4 CONTROL (control qubit in qubits[q_off]),*/
/*   5 ENDCONTROL.                                                     */
/* qubits[q_off[k] ...] lists the targets, then the controls.          */
/* ------------------------------------------------------------------ */

typedef struct {
    int nt, nc;
    int q[2 * OR_MAX_T + 16];
    cplx *m; /* owned, 2^nt x 2^nt */
} or_flat_gate;

typedef struct {
    or_flat_gate *g;
    int count, cap;
} or_flat_list;

static void flat_push(or_flat_list *l, const or_flat_gate *g)
{
    if (l->count == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->g = realloc(l->g, (size_t)l->cap * sizeof(or_flat_gate));
    }
    l->g[l->count++] = *g;
}

static void flat_free(or_flat_list *l)
{
    for (int k = 0; k < l->count; ++k) free(l->g[k].m);
    free(l->g);
    l->g = NULL; l->count = l->cap = 0;
}

/* Find the index of the marker that closes the group opened at `open`. */
static int group_end(const int *kind, int nops, int open)
{
    int depth = 0;
    for (int k = open; k < nops; ++k) {
        if (kind[k] == 2 || kind[k] == 4) ++depth;
        if (kind[k] == 3 || kind[k] == 5) {
            --depth;
            if (depth == 0) return k;
        }
    }
    return -1;
}

/*
 * Expand ops [lo, hi) of a gate-only region into flat gates.  A DAGGER group
 * becomes the reversed list of conjugate-transposed gates; a CONTROL group
 * adds its qubit to the controls of every gate inside.  Returns 0, or -1 on
 * an unbalanced group or a noise site inside a group.
 */
static int expand(const int *kind, const int *nt, const int *nc, const int *q_off,
                  const int *qubits, const int *mat_off, const double *mats,
                  int lo, int hi, or_flat_list *out)
{
    for (int k = lo; k < hi; ++k) {
        if (kind[k] == 0) {
            or_flat_gate g;
            g.nt = nt[k]; g.nc = nc[k];
            if (g.nt < 0 || g.nt > OR_MAX_T || g.nc < 0 || g.nt + g.nc > 2 * OR_MAX_T + 16)
                return -1;
            for (int a = 0; a < g.nt + g.nc; ++a) g.q[a] = qubits[q_off[k] + a];
            int d = 1 << g.nt;
            g.m = malloc((size_t)d * d * sizeof(cplx));
            for (int e = 0; e < d * d; ++e)
                g.m[e] = mats[2 * ((size_t)mat_off[k] + e)] + I * mats[2 * ((size_t)mat_off[k] + e) + 1];
            flat_push(out, &g);
        } else if (kind[k] == 2 || kind[k] == 4) {
            int e = group_end(kind, hi, k);
            if (e < 0) return -1;
            if ((kind[k] == 2) != (kind[e] == 3)) return -1;
            or_flat_list inner = {0};
            if (expand(kind, nt, nc, q_off, qubits, mat_off, mats, k + 1, e, &inner)) {
                flat_free(&inner);
                return -1;
            }
            if (kind[k] == 2) {
                /* DAGGER: (G_1 ... G_m)^dagger = G_m^dagger ... G_1^dagger */
                for (int a = inner.count - 1; a >= 0; --a) {
                    or_flat_gate g = inner.g[a];
                    int d = 1 << g.nt;
                    cplx *mt = malloc((size_t)d * d * sizeof(cplx));
                    for (int r = 0; r < d; ++r)
                        for (int c = 0; c < d; ++c) mt[r * d + c] = conj(g.m[c * d + r]);
                    free(g.m);
                    g.m = mt;
                    flat_push(out, &g);
                }
            } else {
                /* CONTROL i: every gate in the group gains control qubit i */
                int cq = qubits[q_off[k]];
                for (int a = 0; a < inner.count; ++a) {
                    or_flat_gate g = inner.g[a];
                    if (g.nt + g.nc + 1 > 2 * OR_MAX_T + 16) {
                        for (int b = a; b < inner.count; ++b) free(inner.g[b].m);
                        free(inner.g);
                        return -1;
                    }
                    g.q[g.nt + g.nc] = cq;
                    g.nc += 1;
                    flat_push(out, &g);
                }
            }
            free(inner.g);
            k = e;
        } else {
            return -1; /* noise inside a group, or a stray end marker */
        }
    }
    return 0;
}

/*
 * Run an op list on psi (already initialised).  Noise sites draw
 * u = or_uniform(seed, traj, site) with site = 0, 1, 2, ... in order of
 * appearance, and the branch of site s is written to chosen_out[s] if given.
 * Returns 0, or a negative code.
 */
int or_run(cplx *psi, int n, int nops, const int *kind, const int *nt, const int *nc,
           const int *q_off, const int *qubits, const int *mat_off, const double *mats,
           const int *nk, uint64_t seed, uint64_t traj, int *chosen_out)
{
    or_flat_gate prev = {0};
    int have_prev = 0;
    uint64_t site = 0;
    for (int k = 0; k < nops; ++k) {
        if (kind[k] == 1) {
            /* noise after the preceding gate: the noisy gate K_b * U */
            if (!have_prev || prev.nc != 0 || prev.nt != nt[k]) return -3;
            for (int a = 0; a < nt[k]; ++a)
                if (prev.q[a] != qubits[q_off[k] + a]) return -3;
            int d = 1 << nt[k];
            cplx *kr = malloc((size_t)nk[k] * d * d * sizeof(cplx));
            for (size_t e = 0; e < (size_t)nk[k] * d * d; ++e)
                kr[e] = mats[2 * ((size_t)mat_off[k] + e)] + I * mats[2 * ((size_t)mat_off[k] + e) + 1];
            /* undo nothing: the gate was held back and is applied here */
            double u = or_uniform(seed, traj, site);
            int ch; double pc;
            int rc = or_apply_noisy(psi, n, prev.q, prev.nt, prev.m, kr, nk[k], u, &ch, &pc, NULL);
            free(kr);
            if (rc) return rc;
            if (chosen_out) chosen_out[site] = ch;
            ++site;
            free(prev.m);
            have_prev = 0;
            continue;
        }
        /* flush a held-back gate that has no noise site after it */
        if (have_prev) {
            if (or_apply(psi, n, prev.q, prev.nt, prev.q + prev.nt, prev.nc, prev.m)) return -1;
            free(prev.m);
            have_prev = 0;
        }
        if (kind[k] == 0) {
            /* hold the gate back: a noise site may follow it */
            or_flat_list one = {0};
            if (expand(kind, nt, nc, q_off, qubits, mat_off, mats, k, k + 1, &one)) return -1;
            prev = one.g[0];
            free(one.g);
            have_prev = 1;
        } else if (kind[k] == 2 || kind[k] == 4) {
            int e = group_end(kind, nops, k);
            if (e < 0) return -2;
            or_flat_list fl = {0};
            if (expand(kind, nt, nc, q_off, qubits, mat_off, mats, k, e + 1, &fl)) {
                flat_free(&fl);
                return -2;
            }
            for (int a = 0; a < fl.count; ++a) {
                or_flat_gate *g = &fl.g[a];
                if (or_apply(psi, n, g->q, g->nt, g->q + g->nt, g->nc, g->m)) {
                    flat_free(&fl);
                    return -1;
                }
            }
            flat_free(&fl);
            k = e;
        } else {
            return -2;
        }
    }
    if (have_prev) {
        int rc = or_apply(psi, n, prev.q, prev.nt, prev.q + prev.nt, prev.nc, prev.m);
        free(prev.m);
        if (rc) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Fully connected network F -> H -> H -> 1 with ReLU, FP64.            */
/* Parameters, packed one after another:                               */
/*   W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3.                      */
/* Loss = (1/B) sum_s (y_s - t_s)^2.                                   */
/* ------------------------------------------------------------------ */
size_t or_mlp_num_params(int f, int h)
{
    return (size_t)h * f + h + (size_t)h * h + h + h + 1;
}

/* Forward pass for B samples x[B][F]; writes y[B], returns the loss if t
 * is given (else 0) and, if grad != NULL, the gradient of the loss with
 * respect to every parameter. */
double or_mlp_forward_backward(const double *params, int f, int h, int bsz,
                               const double *x, const double *t, double *y, double *grad)
{
    const double *W1 = params, *b1 = W1 + (size_t)h * f, *W2 = b1 + h,
                 *b2 = W2 + (size_t)h * h, *W3 = b2 + h, *b3 = W3 + h;
    size_t np = or_mlp_num_params(f, h);
    double *gW1 = NULL, *gb1 = NULL, *gW2 = NULL, *gb2 = NULL, *gW3 = NULL, *gb3 = NULL;
    if (grad) {
        memset(grad, 0, np * sizeof(double));
        gW1 = grad; gb1 = gW1 + (size_t)h * f; gW2 = gb1 + h;
        gb2 = gW2 + (size_t)h * h; gW3 = gb2 + h; gb3 = gW3 + h;
    }
    double *z1 = malloc((size_t)h * sizeof(double)), *a1 = malloc((size_t)h * sizeof(double));
    double *z2 = malloc((size_t)h * sizeof(double)), *a2 = malloc((size_t)h * sizeof(double));
    double *d2 = malloc((size_t)h * sizeof(double)), *d1 = malloc((size_t)h * sizeof(double));
    double loss = 0.0;
    for (int s = 0; s < bsz; ++s) {
        const double *xs = x + (size_t)s * f;
        for (int j = 0; j < h; ++j) {
            double acc = b1[j];
            for (int k = 0; k < f; ++k) acc += W1[(size_t)j * f + k] * xs[k];
            z1[j] = acc;
            a1[j] = acc > 0 ? acc : 0;
        }
        for (int j = 0; j < h; ++j) {
            double acc = b2[j];
            for (int k = 0; k < h; ++k) acc += W2[(size_t)j * h + k] * a1[k];
            z2[j] = acc;
            a2[j] = acc > 0 ? acc : 0;
        }
        double out = b3[0];
        for (int k = 0; k < h; ++k) out += W3[k] * a2[k];
        if (y) y[s] = out;
        if (t) {
            double e = out - t[s];
            loss += e * e / bsz;
            if (grad) {
                double dy = 2.0 * e / bsz;
                gb3[0] += dy;
                for (int k = 0; k < h; ++k) {
                    gW3[k] += dy * a2[k];
                    d2[k] = z2[k] > 0 ? dy * W3[k] : 0.0;
                }
                for (int j = 0; j < h; ++j) {
                    gb2[j] += d2[j];
                    for (int k = 0; k < h; ++k) gW2[(size_t)j * h + k] += d2[j] * a1[k];
                }
                for (int k = 0; k < h; ++k) {
                    double acc = 0.0;
                    for (int j = 0; j < h; ++j) acc += W2[(size_t)j * h + k] * d2[j];
                    d1[k] = z1[k] > 0 ? acc : 0.0;
                }
                for (int j = 0; j < h; ++j) {
                    gb1[j] += d1[j];
                    for (int k = 0; k < f; ++k) gW1[(size_t)j * f + k] += d1[j] * xs[k];
                }
            }
        }
    }
    free(z1); free(a1); free(z2); free(a2); free(d2); free(d1);
    return loss;
}
