"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each expected value is a
closed form, a value printed in the paper, an independent construction
(Kronecker-product operators), an algebraic identity or a published
known-answer vector.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2008_07140_amd import circuits as cg
from tests import appa_script

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)


# ------------------------------------------------------------------ helpers --


def full_operator(n, targets, controls, m):
    """Dense 2^n operator of a (controlled) gate built from Kronecker products.

    Independent of the oracle's index loop: qubit q is bit q of the index, so
    the Kronecker factor of qubit n-1 is leftmost.  M = sum_ab M_ab |a><b| on
    the targets (targets[0] = most significant bit of a), times the projector
    onto |1> of every control, plus the identity on the complement of that
    projector."""
    dim = 1 << n
    nt = len(targets)

    def kron_all(factors):
        out = np.ones((1, 1), dtype=complex)
        for q in range(n - 1, -1, -1):
            out = np.kron(out, factors.get(q, np.eye(2, dtype=complex)))
        return out

    proj = kron_all({c: P1 for c in controls}) if controls else np.eye(dim, dtype=complex)
    op = np.eye(dim, dtype=complex) - proj
    for a in range(1 << nt):
        for b in range(1 << nt):
            if m[a, b] == 0:
                continue
            f = {c: P1 for c in controls}
            for t_idx, q in enumerate(targets):
                abit = (a >> (nt - 1 - t_idx)) & 1
                bbit = (b >> (nt - 1 - t_idx)) & 1
                e = np.zeros((2, 2), dtype=complex)
                e[abit, bbit] = 1
                f[q] = e
            op = op + m[a, b] * kron_all(f)
    return op


def qft_ops(m):
    """Gate order of the QFT used in App. A-2 (third column), for m qubits:
    for j = m-1 .. 0: H j, then CR(k, j, pi / 2^(j-k)) for k = j-1 .. 0;
    then SWAP(i, m-1-i)."""
    ops = []
    for j in range(m - 1, -1, -1):
        ops.append(("H", (j,), ()))
        for k in range(j - 1, -1, -1):
            ops.append(("CR", (k, j), (math.pi / 2 ** (j - k),)))
    for i in range(m // 2):
        ops.append(("SWAP", (i, m - 1 - i), ()))
    return ops


def run_named(psi, ops):
    for name, qs, params in ops:
        oracle.apply(psi, qs, (), oracle.named_gate(name, params))


# --------------------------------------------------------- closed forms --


@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_hadamard_all_gives_uniform_state(n):
    psi = oracle.zero_state(n)
    h = oracle.named_gate("H")
    for q in range(n):
        oracle.apply(psi, (q,), (), h)
    assert np.allclose(psi, 2 ** (-n / 2), atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [2, 5, 8])
def test_ghz_closed_form_named_cnot_and_controlled_x(n):
    expect = np.zeros(1 << n, dtype=complex)
    expect[0] = expect[-1] = 1 / math.sqrt(2)
    # CNOT as the 4x4 matrix of App. A-1 (first listed = control = MSB)
    psi = oracle.zero_state(n)
    oracle.apply(psi, (0,), (), oracle.named_gate("H"))
    for q in range(n - 1):
        oracle.apply(psi, (q, q + 1), (), oracle.named_gate("CNOT"))
    assert np.allclose(psi, expect, atol=1e-15)
    # the same chain as X with a control (Eq. 3)
    psi = oracle.zero_state(n)
    oracle.apply(psi, (0,), (), oracle.named_gate("H"))
    for q in range(n - 1):
        oracle.apply(psi, (q + 1,), (q,), oracle.named_gate("X"))
    assert np.allclose(psi, expect, atol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_qft_of_basis_states_is_dft(m):
    N = 1 << m
    for x in range(N):
        psi = np.zeros(N, dtype=complex)
        psi[x] = 1
        run_named(psi, qft_ops(m))
        y = np.arange(N)
        expect = np.exp(2j * math.pi * x * y / N) / math.sqrt(N)
        assert np.allclose(psi, expect, atol=1e-13), (m, x)


def test_u4_angles_equal_phase_times_rz_ry_rz():
    rng = np.random.default_rng(7)
    for _ in range(20):
        al, be, ga, de = rng.uniform(-4, 4, size=4)
        u = oracle.named_gate("U4", (al, be, ga, de))
        rzb = np.diag([np.exp(-0.5j * be), np.exp(0.5j * be)])
        rzd = np.diag([np.exp(-0.5j * de), np.exp(0.5j * de)])
        c, s = math.cos(ga / 2), math.sin(ga / 2)
        ryg = np.array([[c, -s], [s, c]])
        assert np.allclose(u, np.exp(1j * al) * rzb @ ryg @ rzd, atol=1e-14)


def test_rotation_gates_are_exponentials_of_paulis():
    """RX, RY, RZ (App. A-1) are rotations about the x, y, z axes,
    exp(-i theta P / 2), with P built from gates pinned elsewhere: X (a basis
    permutation), Z = H X H and Y = i X Z.  A sign error in the printed
    off-diagonal of RX or RY, or in the phases of RZ, fails here."""
    from scipy.linalg import expm
    h, x = oracle.named_gate("H"), oracle.named_gate("X")
    z = h @ x @ h
    y = 1j * x @ z
    assert np.allclose(oracle.named_gate("Z"), z, atol=1e-15)
    assert np.allclose(oracle.named_gate("Y"), y, atol=1e-15)
    for theta in (0.3, -1.7, 2.9, math.pi):
        for name, p in (("RX", x), ("RY", y), ("RZ", z)):
            assert np.allclose(oracle.named_gate(name, (theta,)), expm(-0.5j * theta * p), atol=1e-14), (name, theta)
        # the same rotations related to each other by the basis change H
        assert np.allclose(oracle.named_gate("RX", (theta,)),
                           h @ oracle.named_gate("RZ", (theta,)) @ h, atol=1e-14)


def test_phase_gate_powers():
    """T^2 = S and S^2 = Z: T is the fourth root of Z with the phase e^{+i pi/4}
    on |1> that App. A-1 prints, and S = T^2 its square root."""
    t, s, z = (oracle.named_gate(g) for g in ("T", "S", "Z"))
    assert np.allclose(t @ t, s, atol=1e-15)
    assert np.allclose(s @ s, z, atol=1e-15)
    # and T is diagonal with |1> picking up a phase of +pi/4 (not -pi/4)
    assert abs(t[1, 1] - np.exp(0.25j * math.pi)) < 1e-15 and t[0, 0] == 1


def test_u4_reduces_to_rz_for_zero_gamma():
    """U4(0, theta, 0, 0) = RZ(theta): with gamma = 0 the angle form of App. A-1
    is the z rotation by beta (RZ pinned above as exp(-i theta Z / 2))."""
    for theta in (0.4, -2.2):
        assert np.allclose(oracle.named_gate("U4", (0.0, theta, 0.0, 0.0)),
                           oracle.named_gate("RZ", (theta,)), atol=1e-15)


def test_iswap_as_printed():
    """iSWAP of App. A-1 exchanges |01> and |10> with a factor -i (the printed
    matrix; first listed qubit = most significant bit): on qubits (a, b),
    |a=0, b=1> -> -i |a=1, b=0>, and it equals exp(-i pi/4 (X X + Y Y)) built
    from the pinned Paulis, the sign the paper prints."""
    from scipy.linalg import expm
    h, x = oracle.named_gate("H"), oracle.named_gate("X")
    y = 1j * x @ (h @ x @ h)
    u = oracle.named_gate("ISWAP")
    assert np.allclose(u, expm(-0.25j * math.pi * (np.kron(x, x) + np.kron(y, y))), atol=1e-14)
    n, a, b = 3, 2, 0
    psi = np.zeros(1 << n, dtype=complex)
    psi[1 << b] = 1  # qubit a = 0, qubit b = 1
    oracle.apply(psi, (a, b), (), u)
    want = np.zeros(1 << n, dtype=complex)
    want[1 << a] = -1j
    assert np.allclose(psi, want, atol=1e-15)
    # |00> and |11> are unchanged
    for x0 in (0, (1 << a) | (1 << b)):
        psi = np.zeros(1 << n, dtype=complex)
        psi[x0] = 1
        oracle.apply(psi, (a, b), (), u)
        assert psi[x0] == 1 and np.count_nonzero(psi) == 1


def test_named_gates_are_unitary():
    for name, params in [("H", ()), ("X", ()), ("Y", ()), ("Z", ()), ("S", ()), ("T", ()),
                         ("RX", (0.3,)), ("RY", (1.1,)), ("RZ", (-2.0,)),
                         ("U4", (0.1, 0.2, 0.3, 0.4)), ("CNOT", ()), ("CZ", ()),
                         ("CR", (0.7,)), ("SWAP", ()), ("ISWAP", ()), ("TOFFOLI", ())]:
        u = oracle.named_gate(name, params)
        assert np.allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-14), name


def test_toffoli_and_cnot_are_basis_permutations():
    n = 4
    for x in range(1 << n):
        psi = np.zeros(1 << n, dtype=complex)
        psi[x] = 1
        oracle.apply(psi, (3, 1, 0), (), oracle.named_gate("TOFFOLI"))
        b3, b1, b0 = (x >> 3) & 1, (x >> 1) & 1, x & 1
        y = x ^ (1 if (b3 and b1) else 0)
        assert psi[y] == 1 and np.count_nonzero(psi) == 1
        psi = np.zeros(1 << n, dtype=complex)
        psi[x] = 1
        oracle.apply(psi, (2, 0), (), oracle.named_gate("CNOT"))
        y = x ^ (1 if (x >> 2) & 1 else 0)
        assert psi[y] == 1 and np.count_nonzero(psi) == 1


def test_swap_exchanges_the_values_of_its_qubits():
    """SWAP (App. A-1) on every basis state of 5 qubits and every ordered pair
    moves the value of each qubit to the other: |x> -> |x with bits a, b
    exchanged>, brute force."""
    n = 5
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            for x in range(1 << n):
                psi = np.zeros(1 << n, dtype=complex)
                psi[x] = 1
                oracle.apply(psi, (a, b), (), oracle.named_gate("SWAP"))
                ba, bb = (x >> a) & 1, (x >> b) & 1
                y = x & ~((1 << a) | (1 << b)) | (ba << b) | (bb << a)
                assert psi[y] == 1 and np.count_nonzero(psi) == 1


def test_eq4_cz_decomposition():
    """CZ^{i,j} = P0^i (x) I^j + P1^i (x) Z^j (Eq. 4)."""
    n = 6
    rng = np.random.default_rng(3)
    for i, j in [(0, 1), (4, 2), (5, 0), (1, 3)]:
        psi = cg.random_state(n, int(rng.integers(1 << 30)))
        a = psi.copy()
        oracle.apply(a, (i, j), (), oracle.named_gate("CZ"))
        b = psi.copy()
        oracle.apply(b, (i,), (), P0)
        c = psi.copy()
        oracle.apply(c, (i,), (), P1)
        oracle.apply(c, (j,), (), oracle.named_gate("Z"))
        assert np.allclose(a, b + c, atol=1e-15)


def test_eq4_generalised_to_controlled_and_diagonal_gates():
    """The cut rule of the partial-amplitude mode, checked on the oracle: a
    gate U on targets T with controls C' on the other side equals
    P_rest(C') (x) I + P_ones(C') (x) U (Eq. 4 with the all-ones projector,
    for CNOT, CU3 and a Toffoli with both controls across), and a diagonal D
    with one qubit p on one side equals P_0(p) (x) D_0 + P_1(p) (x) D_1 with
    D_v the diagonal restricted to p = v."""
    n = 6
    rng = np.random.default_rng(12)
    X = oracle.named_gate("X")
    for tgt, ctl, u in [((4,), (1,), X), ((0,), (5,), cg.u3(0.4, 1.1, -0.3)), ((3,), (0, 1), X)]:
        psi = cg.random_state(n, int(rng.integers(1 << 30)))
        a = psi.copy()
        oracle.apply(a, tgt, ctl, u)
        k = len(ctl)
        ones = np.zeros(1 << k)
        ones[-1] = 1
        b = psi.copy()
        oracle.apply(b, ctl, (), np.diag(1 - ones))
        c = psi.copy()
        oracle.apply(c, ctl, (), np.diag(ones))
        oracle.apply(c, tgt, (), u)
        assert np.allclose(a, b + c, atol=1e-14)
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, 8))  # on (p, q1, q2), p the high bit
    psi = cg.random_state(n, 99)
    a = psi.copy()
    oracle.apply(a, (2, 3, 4), (), np.diag(d))
    total = np.zeros_like(psi)
    for v in (0, 1):
        t = psi.copy()
        oracle.apply(t, (2,), (), P1 if v else P0)
        oracle.apply(t, (3, 4), (), np.diag(d[4 * v:4 * v + 4]))
        total += t
    assert np.allclose(a, total, atol=1e-14)


# ----------------------------------------------- dense operators, n <= 10 --


def _random_gate(rng, n):
    nt = int(rng.integers(1, 4))
    nc = int(rng.integers(0, min(3, n - nt) + 1))
    qs = rng.permutation(n)[: nt + nc]
    m = cg.random_unitary(1 << nt, rng)
    return tuple(int(q) for q in qs[:nt]), tuple(int(q) for q in qs[nt:]), m


@pytest.mark.parametrize("n", [3, 5, 7])
def test_random_circuit_matches_dense_operator_product(n):
    rng = np.random.default_rng(100 + n)
    psi = oracle.zero_state(n)
    vec = np.zeros(1 << n, dtype=complex)
    vec[0] = 1
    for _ in range(25):
        t, c, m = _random_gate(rng, n)
        oracle.apply(psi, t, c, m)
        vec = full_operator(n, t, c, m) @ vec
    assert np.allclose(psi, vec, atol=1e-13)


def test_dense_operator_single_gates_n10():
    n = 10
    rng = np.random.default_rng(11)
    for t, c in [((0,), ()), ((9,), (0,)), ((3, 7), ()), ((9, 0), (5,)), ((2, 6, 4), (1, 8))]:
        m = cg.random_unitary(1 << len(t), rng)
        psi = cg.random_state(n, int(rng.integers(1 << 30)))
        expect = full_operator(n, t, c, m) @ psi
        oracle.apply(psi, t, c, m)
        assert np.allclose(psi, expect, atol=1e-13)


def test_invalid_qubits_rejected():
    psi = oracle.zero_state(3)
    with pytest.raises(ValueError):
        oracle.apply(psi, (3,), (), np.eye(2))
    with pytest.raises(ValueError):
        oracle.apply(psi, (1,), (1,), np.eye(2))
    with pytest.raises(ValueError):
        oracle.apply(psi, (0, 0), (), np.eye(4))


# ---------------------------------------------------- DAGGER / CONTROL --


def test_circuit_then_dagger_group_returns_zero_state():
    n, ops = 8, cg.random_circuit(2, 4, 6, seed=42, cu3_prob=0.2)
    full = list(ops) + [cg.Marker("dagger")] + list(ops) + [cg.Marker("enddagger")]
    psi, _ = oracle.run(n, full)
    expect = np.zeros(1 << n, dtype=complex)
    expect[0] = 1
    assert np.allclose(psi, expect, atol=1e-12)


def test_nested_dagger_is_identity_on_the_group():
    n, ops = 6, cg.random_circuit(2, 3, 3, seed=5)
    a, _ = oracle.run(n, ops)
    nested = [cg.Marker("dagger"), cg.Marker("dagger")] + list(ops) + [
        cg.Marker("enddagger"), cg.Marker("enddagger")]
    b, _ = oracle.run(n, nested)
    assert np.allclose(a, b, atol=1e-13)


def test_control_groups_add_controls():
    n = 5
    rng = np.random.default_rng(9)
    u = cg.random_unitary(2, rng)
    v = cg.random_unitary(4, rng)
    psi0 = cg.random_state(n, 77)
    # CONTROL 4 { CONTROL 0 { U on 2 ; V on (1, 3) } }
    ops = [cg.Marker("control", 4), cg.Marker("control", 0), cg.Gate((2,), (), u),
           cg.Gate((1, 3), (), v), cg.Marker("endcontrol"), cg.Marker("endcontrol")]
    a, _ = oracle.run(n, ops, psi=psi0.copy())
    b = full_operator(n, (1, 3), (0, 4), v) @ (full_operator(n, (2,), (0, 4), u) @ psi0)
    assert np.allclose(a, b, atol=1e-13)
    # TOFFOLI = CONTROL i { CONTROL j { X k } }
    t = [cg.Marker("control", 0), cg.Marker("control", 1), cg.Gate((3,), (), cg.PX),
         cg.Marker("endcontrol"), cg.Marker("endcontrol")]
    a, _ = oracle.run(n, t, psi=psi0.copy())
    b = psi0.copy()
    oracle.apply(b, (0, 1, 3), (), oracle.named_gate("TOFFOLI"))
    assert np.allclose(a, b, atol=1e-15)


def test_unbalanced_groups_rejected():
    with pytest.raises(ValueError):
        oracle.run(3, [cg.Marker("dagger"), cg.Gate((0,), (), cg.H_GATE)])
    with pytest.raises(ValueError):
        oracle.run(3, [cg.Marker("control", 1), cg.Gate((0,), (), cg.H_GATE),
                       cg.Marker("enddagger")])


# ------------------------------------------------- App. A-2 worked example --


def test_appendix_a2_worked_example_pmeasure():
    with open(os.path.join(GOLDEN, "appA2_example.txt")) as f:
        n, ops, pm, printed = appa_script.parse(f.read(), oracle.named_gate)
    psi, _ = oracle.run(n, ops)
    probs = oracle.probabilities(psi, pm)
    assert abs(probs.sum() - 1) < 1e-14
    assert np.max(np.abs(probs - printed)) < 1e-6


# ---------------------------------------------------------- probabilities --


def test_pmeasure_order_and_marginals():
    n = 6
    psi = cg.random_state(n, 5)
    p_all = oracle.probabilities(psi, list(range(n - 1, -1, -1)))
    assert np.allclose(p_all, np.abs(psi) ** 2, atol=1e-16)
    # reversed listing = bit-reversed output index
    p_rev = oracle.probabilities(psi, list(range(n)))
    rev = [int(format(i, "0%db" % n)[::-1], 2) for i in range(1 << n)]
    assert np.allclose(p_rev, (np.abs(psi) ** 2)[rev], atol=1e-16)
    # marginal over qubits (4, 1): sum of |psi|^2 over the others
    p = oracle.probabilities(psi, [4, 1])
    a2 = (np.abs(psi) ** 2).reshape([2] * n)  # axis 0 = qubit n-1
    marg = a2.sum(axis=tuple(n - 1 - q for q in range(n) if q not in (4, 1)))
    # remaining axes are (qubit 4, qubit 1) in that order
    assert np.allclose(p, marg.reshape(-1), atol=1e-15)
    assert abs(p.sum() - 1) < 1e-14


def test_norm_preserved_by_random_circuit():
    n, ops = 10, cg.random_circuit(2, 5, 8, seed=17, cu3_prob=0.1)
    psi, _ = oracle.run(n, ops)
    assert abs(oracle.norm2(psi) - 1) < 1e-13


# ------------------------------------------------------------ Kraus sets --


@pytest.mark.parametrize("name", sorted(cg.KRAUS_SETS))
@pytest.mark.parametrize("p", [0.0, 0.013, 0.5, 1.0])
def test_kraus_completeness(name, p):
    ks = cg.KRAUS_SETS[name](p)
    s = sum(k.conj().T @ k for k in ks)
    assert np.allclose(s, np.eye(2), atol=1e-15)


def test_kraus_completeness_two_qubit_products():
    for a in cg.KRAUS_SETS.values():
        for b in cg.KRAUS_SETS.values():
            ks = cg.kraus_kron(a(0.2), b(0.07))
            s = sum(k.conj().T @ k for k in ks)
            assert np.allclose(s, np.eye(4), atol=1e-15)


def _dm_of(psi):
    return np.outer(psi, psi.conj())


def test_kraus_special_cases_on_density_matrix():
    n = 3
    psi = cg.random_state(n, 1)
    rho0 = _dm_of(psi)
    for name, p in [("bit_flip", 1.0), ("phase_flip", 1.0), ("bit_phase_flip", 1.0),
                    ("amplitude_damping", 0.0), ("phase_damping", 0.0),
                    ("depolarizing", 0.0)]:
        rho = rho0.copy()
        oracle.dm_channel(rho, (1,), cg.KRAUS_SETS[name](p))
        assert np.allclose(rho, rho0, atol=1e-15), name
    # depolarizing p=1 maps the qubit to I/2: <Z> = 0 there, others unchanged
    rho = rho0.copy()
    oracle.dm_channel(rho, (2,), cg.kraus_depolarizing(1.0))
    z0, z1 = oracle.dm_expect_z(rho0), oracle.dm_expect_z(rho)
    assert abs(z1[2]) < 1e-15 and np.allclose(z1[:2], z0[:2], atol=1e-15)
    # amplitude damping gamma=1 resets the qubit to |0>
    rho = rho0.copy()
    oracle.dm_channel(rho, (0,), cg.kraus_amplitude_damping(1.0))
    assert abs(oracle.dm_expect_z(rho)[0] - 1) < 1e-15


def test_dm_unitary_evolution_matches_pure_state():
    n, ops = 4, cg.random_circuit(2, 2, 6, seed=8, cu3_prob=0.3)
    psi, _ = oracle.run(n, ops)
    rho = oracle.dm_run(n, ops)
    assert np.allclose(rho, _dm_of(psi), atol=1e-13)


# ---------------------------------------------------------- noisy gates --


def test_noisy_gate_depolarizing_branch_probabilities_and_boundaries():
    n, p = 4, 0.2
    psi0 = cg.random_state(n, 12)
    ks = cg.kraus_depolarizing(p)
    u3 = cg.u3(0.3, 1.2, -0.4)
    # state-independent branch weights 1-3p/4, p/4, p/4, p/4
    w = np.array([1 - 3 * p / 4, p / 4, p / 4, p / 4])
    cum = np.cumsum(w)
    for u, expect in [(0.0, 0), (cum[0] - 1e-9, 0), (cum[0] + 1e-9, 1),
                      (cum[1] + 1e-9, 2), (cum[2] + 1e-9, 3), (1 - 1e-12, 3)]:
        psi = psi0.copy()
        ch, pc, probs = oracle.apply_noisy(psi, (2,), u3, ks, u)
        assert np.allclose(probs, w, atol=1e-14)
        assert ch == expect, (u, ch)
        # the result is the normalised (K_b U) psi
        ref = psi0.copy()
        oracle.apply(ref, (2,), (), ks[expect] @ u3)
        ref /= np.linalg.norm(ref)
        assert np.allclose(psi, ref, atol=1e-14)


def test_noisy_gate_amplitude_damping_uses_post_gate_state():
    """|0> -> X -> damping: the post-gate state is |1>, so p(K_2) = gamma.
    (With the pre-gate state it would be 0.)"""
    g = 0.3
    psi = oracle.zero_state(1)
    ch, pc, probs = oracle.apply_noisy(psi, (0,), cg.PX, cg.kraus_amplitude_damping(g), 0.9)
    assert np.allclose(probs, [1 - g, g], atol=1e-15)
    assert ch == 1 and np.allclose(psi, [1, 0], atol=1e-15)


def test_trajectory_mean_matches_density_matrix():
    n = 4
    ops = cg.random_circuit(2, 2, 5, seed=21, dep1=0.05, dep2=0.05, damping=0.05)
    rho = oracle.dm_run(n, ops)
    zdm = oracle.dm_expect_z(rho)
    T = 3000
    zs = np.zeros((T, n))
    for t in range(T):
        psi, _ = oracle.run(n, ops, seed=123, traj=t)
        zs[t] = oracle.expect_z(psi)
    mean = zs.mean(axis=0)
    sigma = np.maximum(zs.std(axis=0), 1e-3)
    assert np.all(np.abs(mean - zdm) < 5 * sigma / math.sqrt(T)), (mean, zdm)


# ----------------------------------------------------------------- Philox --


def test_philox_known_answers():
    """Known-answer vectors published with the Random123 library."""
    assert oracle.philox4x32_10([0, 0, 0, 0], [0, 0]) == [
        0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert oracle.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert oracle.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_uniform_in_unit_interval_and_mean():
    us = np.array([oracle.uniform(99, t, s) for t in range(50) for s in range(200)])
    assert us.min() >= 0 and us.max() < 1
    assert abs(us.mean() - 0.5) < 5 * math.sqrt(1 / 12 / us.size)


# -------------------------------------------------------------------- MLP --


def test_mlp_forward_closed_form_and_gradient_finite_differences():
    f, h = 5, 6
    npar = oracle.mlp_num_params(f, h)
    assert npar == h * f + h + h * h + h + h + 1
    # closed form: a single path x0 -> unit 0 -> unit 0 -> output
    params = np.zeros(npar)
    W1 = params[: h * f].reshape(h, f)
    W1[0, 0] = 2.0
    off = h * f + h
    W2 = params[off: off + h * h].reshape(h, h)
    W2[0, 0] = 3.0
    params[off + h * h + h + 0] = 0.5  # W3[0]
    params[-1] = -1.0  # b3
    x = np.array([[1.5, 9, 9, 9, 9], [-2.0, 0, 0, 0, 0]])
    y, _, _ = oracle.mlp_forward_backward(params, f, h, x)
    assert np.allclose(y, [0.5 * 3 * 2 * 1.5 - 1.0, -1.0], atol=0)
    # gradient vs central differences on random parameters
    rng = np.random.default_rng(0)
    params = rng.standard_normal(npar) * 0.5
    x = rng.standard_normal((7, f))
    t = rng.standard_normal(7)
    _, loss, grad = oracle.mlp_forward_backward(params, f, h, x, t)
    eps = 1e-6
    for k in rng.choice(npar, 40, replace=False):
        pp, pm = params.copy(), params.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (oracle.mlp_forward_backward(pp, f, h, x, t)[1]
              - oracle.mlp_forward_backward(pm, f, h, x, t)[1]) / (2 * eps)
        assert abs(fd - grad[k]) < 1e-6 * max(1, abs(fd)), k
