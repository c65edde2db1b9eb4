"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

complex128: max |delta amp| <= 1e-12 (element by element).
complex64: infidelity <= 1e-5 and max |delta amp| <= 2e-5 after a few gates.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2008_07140_amd import circuits as cg
from tests import appa_script

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL128 = 1e-12


@pytest.fixture(scope="module")
def qs():
    from paper_2008_07140_amd import qs as mod
    return mod


def infidelity(a, b):
    ov = abs(np.vdot(a, b)) ** 2
    return 1 - ov / (np.vdot(a, a).real * np.vdot(b, b).real)


def random_gate(rng, n, nt, nc):
    qs_ = rng.permutation(n)[: nt + nc]
    return (tuple(int(q) for q in qs_[:nt]), tuple(int(q) for q in qs_[nt:]),
            cg.random_unitary(1 << nt, rng))


# ------------------------------------------------------------ single gates --


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nt", [1, 2, 3, 4, 5, 6])
def test_dense_gates_match_oracle(qs, dtype, nt):
    n = 13
    rng = np.random.default_rng(1000 + nt)
    dt = qs.C128 if dtype == "c128" else qs.C64
    s = qs.State(n, dt)
    psi = cg.random_state(n, 3 + nt)
    s.set_amplitudes(psi)
    ref = psi.copy()
    for trial in range(6):
        nc = trial % 3
        t, c, m = random_gate(rng, n, nt, nc)
        if trial == 0:  # include the extreme positions
            t = tuple([n - 1] + list(t[1:])) if n - 1 not in c else t
            if 0 not in t and 0 not in c:
                t = tuple(list(t[:-1]) + [0]) if nt > 1 else t
        s.apply_gate(t, c, m)
        oracle.apply(ref, t, c, m)
    got = s.amplitudes()
    if dtype == "c128":
        assert np.max(np.abs(got - ref)) <= TOL128
    else:
        assert infidelity(ref, got) <= 1e-5
        assert np.max(np.abs(got - ref)) <= 2e-5
    s.close()


@pytest.mark.parametrize("target", [0, 1, 2, 3, 5, 8, 15, 16])
def test_one_qubit_every_position_with_controls(qs, target):
    n = 17
    rng = np.random.default_rng(target)
    s = qs.State(n, qs.C128)
    psi = cg.random_state(n, 50 + target)
    s.set_amplitudes(psi)
    ref = psi.copy()
    for controls in [(), ((target + 1) % n,), ((target + 3) % n, (target + 7) % n)]:
        m = cg.random_unitary(2, rng)
        s.apply_gate((target,), controls, m)
        oracle.apply(ref, (target,), controls, m)
    assert np.max(np.abs(s.amplitudes() - ref)) <= TOL128


def test_diagonal_and_controlled_forms(qs):
    n = 11
    rng = np.random.default_rng(5)
    s = qs.State(n, qs.C128)
    psi = cg.random_state(n, 9)
    s.set_amplitudes(psi)
    ref = psi.copy()
    gates = [
        ((3,), (), cg.T_GATE), ((0,), (), cg.rz(0.7)), ((10,), (), cg.PZ),
        ((2, 7), (), cg.CZ_GATE), ((7, 2), (), cg.CZ_GATE), ((0, 1), (), cg.CZ_GATE),
        ((4, 9), (), oracle.named_gate("CR", (0.3,))), ((9, 4), (), oracle.named_gate("CNOT")),
        ((1, 5, 8), (), oracle.named_gate("TOFFOLI")), ((6,), (2, 3), cg.PX),
        ((5,), (), np.eye(2)), ((5, 6), (), np.diag(np.exp(1j * rng.uniform(0, 6, 4)))),
        (tuple(range(6)), (), np.diag(np.exp(1j * rng.uniform(0, 6, 64)))),
        ((3, 8), (), oracle.named_gate("SWAP")), ((2, 9), (), oracle.named_gate("ISWAP")),
        ((4,), (), -np.eye(2)),  # global phase
    ]
    for t, c, m in gates:
        s.apply_gate(t, c, m)
        oracle.apply(ref, t, c, m)
        got = s.amplitudes()
        assert np.max(np.abs(got - ref)) <= TOL128, (t, c)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gates_on_the_lowest_qubits_whole_runs(qs, dtype):
    """Diagonal gates with a qubit inside the 128-byte run (bits 0-2 of
    complex128, 0-3 of complex64) and single-target gates with such a
    control and the target above it move whole runs and change only the
    selected amplitudes: every form against the oracle, on 12 qubits."""
    n = 12
    rng = np.random.default_rng(31)
    dt = qs.C128 if dtype == "c128" else qs.C64
    s = qs.State(n, dt)
    psi = cg.random_state(n, 33)
    s.set_amplitudes(psi)
    ref = psi.copy()
    gates = [
        ((0, 1), (), cg.CZ_GATE), ((2, 9), (), cg.CZ_GATE), ((11, 3), (), cg.CZ_GATE),
        ((1,), (), cg.T_GATE), ((0,), (), cg.rz(0.4)), ((3,), (), cg.T_GATE),
        ((1, 2), (), oracle.named_gate("CR", (0.9,))), ((0, 1, 2), (), oracle.named_gate("TOFFOLI")),
        ((5,), (1,), cg.u3(0.3, 0.8, -1.1)), ((7,), (0, 2), cg.u3(1.3, -0.2, 0.5)),
        ((4,), (3,), cg.u3(0.6, 0.1, 0.9)), ((10,), (2, 8), cg.random_unitary(2, rng)),
        ((6,), (0,), cg.PZ),
    ]
    tol = TOL128 if dt == qs.C128 else 2e-6
    for t, c, m in gates:
        s.apply_gate(t, c, m)
        oracle.apply(ref, t, c, m)
        got = s.amplitudes()
        assert np.max(np.abs(got - ref)) <= tol, (t, c)
    s.close()


def test_edge_sizes(qs):
    # n = 1, gate on every qubit of the state, controls on all others
    for n in [1, 2, 6]:
        rng = np.random.default_rng(n)
        s = qs.State(n, qs.C128)
        psi = cg.random_state(n, n)
        s.set_amplitudes(psi)
        ref = psi.copy()
        nt = min(n, 6)
        m = cg.random_unitary(1 << nt, rng)
        t = tuple(range(nt))[::-1]
        s.apply_gate(t, (), m)
        oracle.apply(ref, t, (), m)
        if n > 1:
            m1 = cg.random_unitary(2, rng)
            s.apply_gate((0,), tuple(range(1, n)), m1)
            oracle.apply(ref, (0,), tuple(range(1, n)), m1)
        assert np.max(np.abs(s.amplitudes() - ref)) <= TOL128


def test_invalid_gate_leaves_state_unchanged(qs):
    s = qs.State(5, qs.C128)
    psi = cg.random_state(5, 2)
    s.set_amplitudes(psi)
    with pytest.raises(qs.QSError):
        s.apply_gate((5,), (), cg.H_GATE)
    with pytest.raises(qs.QSError):
        s.apply_gate((1,), (1,), cg.H_GATE)
    with pytest.raises(qs.QSError):
        s.apply_noisy_gate((1,), cg.H_GATE, cg.kraus_depolarizing(0.1), 1.5)
    assert np.max(np.abs(s.amplitudes() - psi)) == 0


# -------------------------------------------------------------- reductions --


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_reductions(qs, dtype):
    n = 14
    dt = qs.C128 if dtype == "c128" else qs.C64
    s = qs.State(n, dt)
    psi = cg.random_state(n, 77)
    s.set_amplitudes(psi)
    ref = s.amplitudes()  # the stored (possibly rounded) state, exactly as doubles
    assert abs(s.norm() - np.vdot(ref, ref).real) < 1e-13
    for qubits in [[0], [13], [5, 2], [0, 13, 7], [1, 3, 5, 7, 9], list(range(11)),
                   list(range(12, -1, -1)), None]:
        got = s.probabilities(qubits)
        want = oracle.probabilities(ref, qubits if qubits is not None else list(range(n - 1, -1, -1)))
        assert np.max(np.abs(got - want)) < 1e-13, qubits
    z = s.expect_z()
    assert np.max(np.abs(z - oracle.expect_z(ref))) < 1e-12
    rng = np.random.default_rng(0)
    idx = rng.choice(1 << n, 500, replace=False).astype(np.uint64)
    assert np.array_equal(s.amplitudes(idx), ref[idx])


def test_appendix_a2_worked_example_on_gpu(qs):
    with open(os.path.join(GOLDEN, "appA2_example.txt")) as f:
        n, ops, pm, printed = appa_script.parse(f.read(), oracle.named_gate)
    s = qs.State(n, qs.C128)
    s.run(qs.Circuit(ops))
    probs = s.probabilities(pm)
    assert np.max(np.abs(probs - printed)) < 1e-6
    psi, _ = oracle.run(n, ops)
    assert np.max(np.abs(s.amplitudes() - psi)) <= TOL128


# ------------------------------------------------------------------ circuits --


@pytest.mark.parametrize("plan,kmax", [(0, 0), (1, 2), (1, 3), (1, 4), (1, 5), (1, 6)])
def test_rqc16_depth20_full_vector(qs, plan, kmax):
    n, ops = cg.workload("rqc16_d20")
    ref, _ = oracle.run(n, ops)
    s = qs.State(n, qs.C128)
    s.run(qs.Circuit(ops), plan=plan, k_max=kmax)
    got = s.amplitudes()
    assert np.max(np.abs(got - ref)) <= TOL128
    p = s.probabilities()
    assert np.max(np.abs(p - np.abs(ref) ** 2)) <= 1e-14
    s.close()


@pytest.mark.parametrize("plan,kmax", [(0, 0), (1, 4), (1, 6)])
def test_rqc_c64_infidelity(qs, plan, kmax):
    rows, cols, depth = 4, 5, 40
    ops = cg.random_circuit(rows, cols, depth, seed=2001, cu3_prob=0.1)
    n = rows * cols
    ref, _ = oracle.run(n, ops)
    s = qs.State(n, qs.C64)
    s.run(qs.Circuit(ops), plan=plan, k_max=kmax)
    got = s.amplitudes()
    assert infidelity(ref, got) <= 1e-5


def test_groups_dagger_control(qs):
    n, ops = 9, cg.random_circuit(2, 4, 5, seed=3, cu3_prob=0.3)  # gates on qubits 0..7
    full = ([cg.Marker("control", 8)] + list(ops[:20]) + [cg.Marker("endcontrol")]
            + [cg.Marker("dagger")] + list(ops) + [cg.Marker("control", 8)] + list(ops[:9])
            + [cg.Marker("endcontrol"), cg.Marker("enddagger")])
    ref, _ = oracle.run(n, full)
    s = qs.State(n, qs.C128)
    s.set_amplitudes(cg.random_state(n, 1))
    s.reset()
    s.run(qs.Circuit(full))
    assert np.max(np.abs(s.amplitudes() - ref)) <= TOL128


# ------------------------------------------------------------------- noise --


def test_noisy_gate_matches_oracle_branch_and_state(qs):
    n = 8
    rng = np.random.default_rng(4)
    psi = cg.random_state(n, 4)
    cases = [((3,), cg.u3(0.4, 1.0, 2.0), cg.kraus_depolarizing(0.3)),
             ((0,), cg.SQRT_X, cg.kraus_amplitude_damping(0.4)),
             ((7,), cg.H_GATE, cg.kraus_phase_damping(0.5)),
             ((2,), cg.T_GATE, cg.kraus_bit_flip(0.6)),
             ((1, 6), cg.CZ_GATE, cg.kraus_kron(cg.kraus_depolarizing(0.2), cg.kraus_depolarizing(0.3))),
             ((5, 4), cg.random_unitary(4, rng), cg.kraus_kron(cg.kraus_amplitude_damping(0.3),
                                                               cg.kraus_phase_flip(0.7)))]
    for t, m, ks in cases:
        for u in [0.01, 0.35, 0.62, 0.97]:
            s = qs.State(n, qs.C128)
            s.set_amplitudes(psi)
            ch, pc = s.apply_noisy_gate(t, m, ks, u)
            ref = psi.copy()
            och, opc, _ = oracle.apply_noisy(ref, t, m, ks, u)
            assert ch == och, (t, u)
            assert abs(pc - opc) < 1e-12
            assert np.max(np.abs(s.amplitudes() - ref)) <= TOL128
            s.close()


def test_noisy_circuit_matches_oracle_trajectories(qs):
    n = 8
    ops = cg.random_circuit(2, 4, 6, seed=31, dep1=0.05, dep2=0.05, damping=0.05)
    nsites = sum(1 for o in ops if o.kind == "noise")
    c = qs.Circuit(ops)
    s = qs.State(n, qs.C128)
    for traj in range(6):
        s.reset()
        chosen = s.run(c, seed=77, traj=traj, nsites=nsites)
        ref, och = oracle.run(n, ops, seed=77, traj=traj)
        assert np.array_equal(chosen, och)
        assert np.max(np.abs(s.amplitudes() - ref)) <= TOL128


# -------------------------------------------------------- full-size checks --


def test_rqc30_depth40_c128_full_size_properties(qs):
    """At the benchmark size: norm preserved, and the circuit followed by its
    DAGGER group returns |0...0> (any index error or dropped term breaks it)."""
    n, ops = cg.workload("rqc30_d40")
    s = qs.State(n, qs.C128)
    s.run(qs.Circuit(ops))
    assert abs(s.norm() - 1) < 1e-10
    inv = [cg.Marker("dagger")] + list(ops) + [cg.Marker("enddagger")]
    s.run(qs.Circuit(inv))
    a = s.amplitudes(np.array([0, 1, 2, 1 << 29, (1 << 30) - 1], dtype=np.uint64))
    assert abs(a[0] - 1) < 1e-10 and np.max(np.abs(a[1:])) < 1e-10
    s.close()


def _product_circuit(half_a, half_b, nh):
    """Two independent nh-qubit circuits placed on the even and the odd qubits
    of a 2*nh-qubit register, interleaved gate by gate."""
    def remap(ops, f):
        return [cg.Gate(tuple(f(q) for q in o.targets), tuple(f(q) for q in o.controls),
                        o.matrix, o.name) for o in ops]

    ev = remap(half_a, lambda q: 2 * q)
    od = remap(half_b, lambda q: 2 * q + 1)
    return [g for pair in zip(ev, od) for g in pair] + ev[len(od):] + od[len(ev):]


def _product_expected(half_a, half_b, nh, idx):
    """Each amplitude of the product state is a_even(bits 0,2,4..) times
    a_odd(bits 1,3,5..), both from the oracle on nh qubits."""
    a_ev, _ = oracle.run(nh, half_a)
    a_od, _ = oracle.run(nh, half_b)
    ev_idx = np.zeros(idx.size, dtype=np.int64)
    od_idx = np.zeros(idx.size, dtype=np.int64)
    for b in range(nh):
        ev_idx |= ((idx >> np.uint64(2 * b)) & np.uint64(1)).astype(np.int64) << b
        od_idx |= ((idx >> np.uint64(2 * b + 1)) & np.uint64(1)).astype(np.int64) << b
    return a_ev[ev_idx] * a_od[od_idx]


def _sample_indices(n, count, seed, forced):
    rng = np.random.default_rng(seed)
    idx = rng.choice(1 << n, count, replace=False).astype(np.uint64)
    idx[: len(forced)] = np.array(forced, dtype=np.uint64)
    return idx


def _check_c64_sample(got, want):
    """complex64 bar on a sample: infidelity of the sampled sub-vector
    <= 1e-5 (the bound on the whole state) and every error small against
    the sample's RMS amplitude."""
    assert infidelity(want, got) <= 1e-5
    rms = math.sqrt(float(np.mean(np.abs(want) ** 2)))
    assert np.max(np.abs(got - want)) <= 1e-2 * rms


def test_rqc30_product_circuit_sampled_amplitudes(qs):
    """A 30-qubit circuit made of two independent 15-qubit random circuits on
    the even and the odd qubits: each amplitude is the product of two oracle
    amplitudes, so 2^16 sampled outputs of the full-size launch are checked."""
    half = cg.random_circuit(5, 3, 12, seed=909, cu3_prob=0.1)
    half2 = cg.random_circuit(3, 5, 12, seed=910, cu3_prob=0.1)
    ops = _product_circuit(half, half2, 15)
    idx = _sample_indices(30, 1 << 16, 1, [0, 1, (1 << 30) - 1, 1 << 29])
    want = _product_expected(half, half2, 15, idx)
    for dt, plan, kmax, tol in [(qs.C128, 0, 0, TOL128), (qs.C64, 1, 5, 2e-6), (qs.C128, 1, 3, TOL128)]:
        s = qs.State(30, dt)
        s.run(qs.Circuit(ops), plan=plan, k_max=kmax)
        got = s.amplitudes(idx)
        assert np.max(np.abs(got - want)) <= tol
        s.close()


@pytest.mark.parametrize("m", [12, 13])
def test_tile_sweeps_24_qubits_full_vector(qs, m):
    """24 qubits, 2^11 or 2^12 tiles of 4-qubit blocks (more tiles than the
    compute units hold at once): every amplitude is checked against the
    product of two 12-qubit oracle states, under two tile orders."""
    nh, n = 12, 24
    half = cg.random_circuit(3, 4, 14, seed=1201, cu3_prob=0.1)
    half2 = cg.random_circuit(4, 3, 14, seed=1202, cu3_prob=0.1)
    ops = _product_circuit(half, half2, nh)
    want = _product_expected(half, half2, nh, np.arange(1 << n, dtype=np.uint64))
    c = qs.Circuit(ops)
    info = c.plan_info(n, qs.C64, qs.PLAN_GREEDY, k_max=4, tile_qubits=m)
    assert info["sweeps"] > 1
    s = qs.State(n, qs.C64)
    for order in (1, 3):
        s.reset()
        s.run(c, plan=qs.PLAN_GREEDY, k_max=4, tile_qubits=m, tile_order=order)
        got = s.amplitudes()
        assert infidelity(want, got) <= 1e-6, order
        assert np.max(np.abs(got - want)) <= 1e-5, order
    s.close()


@pytest.mark.parametrize("nh,grid", [(16, (4, 4)), (17, (17, 1))])
def test_product_circuit_above_30_qubits_sampled_amplitudes(qs, nh, grid):
    """32 and 34 qubits (states of 32 and 128 GiB as complex64) through the
    tile path in the benchmark's launch configuration (13-qubit tiles, 4-qubit
    blocks, greedy plan): at 34 qubits there are 2^21 tiles, more than the
    launch grid, so each workgroup walks several tiles; indices at and above
    2^32 are forced into the 2^16-index sample.  The expected values are
    products of two oracle amplitudes on nh qubits.  At 32 qubits the plain
    complex128 path is checked as well (64 GiB)."""
    n = 2 * nh
    half = cg.random_circuit(grid[0], grid[1], 12, seed=950 + nh, cu3_prob=0.1)
    half2 = cg.random_circuit(grid[0], grid[1], 12, seed=970 + nh, cu3_prob=0.1)
    ops = _product_circuit(half, half2, nh)
    top = (1 << n) - 1
    forced = [0, 1, top, 1 << 31, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, top ^ (1 << 32),
              (1 << (n - 1)) | 5, top >> 1, top ^ (1 << 31)]
    forced = sorted(set(f for f in forced if f <= top))
    idx = _sample_indices(n, 1 << 16, 3 + nh, forced)
    want = _product_expected(half, half2, nh, idx)
    print("[product] n=%d c64 greedy tile_qubits=13 k_max=4" % n, flush=True)
    s = qs.State(n, qs.C64)
    c = qs.Circuit(ops)
    info = c.plan_info(n, qs.C64, qs.PLAN_GREEDY, k_max=4, tile_qubits=13)
    assert info["sweeps"] > 1
    s.run(c, plan=qs.PLAN_GREEDY, k_max=4, tile_qubits=13)
    got = s.amplitudes(idx)
    # a split-bfloat16 block (hi + lo operands, about 16 significant bits)
    # is unitary to about 2^-16, so the squared norm may drift by about that
    # much per fused block of the plan
    assert abs(s.norm() - 1) < info["blocks"] * 2.0 ** -16
    s.close()
    _check_c64_sample(got, want)
    if n == 32:
        print("[product] n=32 c128 unfused", flush=True)
        s = qs.State(n, qs.C128)
        s.run(c, plan=qs.PLAN_UNFUSED)
        got = s.amplitudes(idx)
        s.close()
        assert np.max(np.abs(got - want)) <= TOL128


# ------------------------------------------------------------ tile sweeps --


def _mixed_circuit(n, count, seed):
    """Random gates of every shape the planner distinguishes: dense 1-3
    targets, controls (which land inside or outside a tile), diagonal gates
    on up to 4 qubits, and an occasional 6-target dense gate (too wide for a
    tile, applied on its own)."""
    rng = np.random.default_rng(seed)
    ops = []
    for i in range(count):
        kind = rng.integers(0, 6)
        if kind == 0:
            t, c, m = random_gate(rng, n, 1, 0)
        elif kind == 1:
            t, c, m = random_gate(rng, n, 1, int(rng.integers(1, 3)))
        elif kind == 2:
            t, c, m = random_gate(rng, n, 2, int(rng.integers(0, 2)))
        elif kind == 3:
            t, c, m = random_gate(rng, n, 3, 0)
        elif kind == 4:
            nt = int(rng.integers(1, 5))
            q = rng.permutation(n)[:nt]
            t, c = tuple(int(x) for x in q), ()
            m = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << nt)))
        else:
            if i % 17 == 0:
                t, c, m = random_gate(rng, n, 6, 0)
            else:
                a, b = (int(x) for x in rng.permutation(n)[:2])
                t, c, m = (a, b), (), cg.CZ_GATE
        ops.append(cg.Gate(t, c, m))
    return ops


@pytest.mark.parametrize("m,kmax", [(10, 4), (11, 5), (12, 4), (13, 5)])
def test_tile_sweeps_c64_mixed_gates(qs, m, kmax):
    n = 14
    ops = _mixed_circuit(n, 160, seed=100 + m)
    ref, _ = oracle.run(n, ops)
    s = qs.State(n, qs.C64)
    info = qs.Circuit(ops).plan_info(n, qs.C64, plan=1, k_max=kmax, tile_qubits=m)
    assert info["sweeps"] < 160
    s.run(qs.Circuit(ops), plan=1, k_max=kmax, tile_qubits=m)
    got = s.amplitudes()
    assert infidelity(ref, got) <= 1e-6
    assert np.max(np.abs(got - ref)) <= 1e-5


@pytest.mark.parametrize("m", [10, 11, 13])
def test_tile_sweeps_rqc16_and_rqc20(qs, m):
    for name, (rows, cols, depth, seed, cu3) in [("rqc16", (4, 4, 20, 1001, 0.0)),
                                                  ("rqc20", (4, 5, 40, 2001, 0.1))]:
        ops = cg.random_circuit(rows, cols, depth, seed, cu3_prob=cu3)
        n = rows * cols
        ref, _ = oracle.run(n, ops)
        s = qs.State(n, qs.C64)
        s.run(qs.Circuit(ops), plan=1, k_max=5, tile_qubits=m)
        got = s.amplitudes()
        assert infidelity(ref, got) <= 1e-6, name
        assert abs(s.norm() - 1) < 1e-4
        s.close()


@pytest.mark.parametrize("m", [10, 13])
def test_tile_orders_give_identical_states(qs, m):
    """The order in which a sweep visits its tiles changes no amplitude: every
    fixed candidate order, and the measured per-sweep choice through its
    timing runs and after them, give bit-identical states (each tile is
    loaded, transformed and stored on its own), equal to the oracle."""
    rows, cols, depth, seed = 4, 5, 12, 777
    ops = cg.random_circuit(rows, cols, depth, seed, cu3_prob=0.1)
    n = rows * cols
    c = qs.Circuit(ops)
    s = qs.State(n, qs.C64)
    outs = []
    for order in list(range(1, qs.TILE_ORDERS + 1)) + [0] * (qs.TILE_ORDERS + 2):
        s.reset()
        s.run(c, plan=qs.PLAN_GREEDY, k_max=4, tile_qubits=m, tile_order=order)
        outs.append(s.amplitudes())
    for i, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), i
    ref, _ = oracle.run(n, ops)
    assert infidelity(ref, outs[0]) <= 1e-6
    with pytest.raises(qs.QSError):
        s.run(c, plan=qs.PLAN_GREEDY, tile_order=qs.TILE_ORDERS + 1)
    s.close()


def test_tile_sweeps_wide_diagonals(qs):
    """Diagonal gates wider than a tile op may be (more than k_max qubits
    inside the tile, or outside qubits beyond the selector limit) run on
    their own between sweeps."""
    n = 20
    rng = np.random.default_rng(9)
    ops = []
    for qubits in [(0, 1, 2, 3, 4, 5), (14, 15, 16, 17, 18, 19), (2, 9, 14, 15, 18, 19)]:
        for q in range(n):
            ops.append(cg.Gate((q,), (), cg.random_unitary(2, rng)))
        ops.append(cg.Gate(qubits, (), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 64)))))
    ref, _ = oracle.run(n, ops)
    for m, k in [(13, 5), (10, 4)]:
        s = qs.State(n, qs.C64)
        s.run(qs.Circuit(ops), plan=1, k_max=k, tile_qubits=m)
        got = s.amplitudes()
        assert infidelity(ref, got) <= 1e-6, (m, k)
        s.close()


def test_tile_sweeps_with_noise_segments(qs):
    """Noise sites split the circuit into segments; each segment is tiled."""
    n = 10
    ops = cg.random_circuit(2, 5, 6, seed=41, dep1=0.05, dep2=0.05, damping=0.05)
    nsites = sum(1 for o in ops if o.kind == "noise")
    c = qs.Circuit(ops)
    s = qs.State(n, qs.C64)
    for traj in range(3):
        s.reset()
        chosen = s.run(c, plan=1, k_max=5, tile_qubits=10, seed=5, traj=traj, nsites=nsites)
        ref, och = oracle.run(n, ops, seed=5, traj=traj)
        assert np.array_equal(chosen, och)
        assert infidelity(ref, s.amplitudes()) <= 1e-6


# ------------------------------------------------------ batched trajectories --


def _traj_batch(count, nmin, nmax, depth, seed, rate):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        r, c = cg.grid_shape(n)
        out.append((n, cg.random_circuit(r, c, depth, seed + t, dep1=rate, dep2=rate, damping=rate)))
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batched_trajectories_match_oracle_per_trajectory(qs, dtype):
    """Each trajectory of the batch is the oracle's literal Sec. 2.4 run with
    the same Philox draws (site s of trajectory t), compared through <Z_q>."""
    batch = _traj_batch(12, 8 if dtype == "c128" else 10, 12, 5, 700, 0.05)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    dt = qs.C128 if dtype == "c128" else qs.C64
    z, sec = qs.run_trajectories(circs, widths, dtype=dt, seed=31)
    off = 0
    for t, (n, ops) in enumerate(batch):
        psi, _ = oracle.run(n, ops, seed=31, traj=t)
        zr = oracle.expect_z(psi)
        tol = 1e-10 if dtype == "c128" else 1e-4
        assert np.max(np.abs(z[off:off + n] - zr)) <= tol, (t, n)
        off += n


def test_trajectory_passes_graph_direct_and_host_sampled_agree(qs):
    """At amplified rates many trajectories jump, so the device-sampled path
    needs several passes (each jump rewrites the trajectory from that site
    on).  The captured-graph passes and the same launches enqueued directly
    give bit-identical results; the host-sampled path (per-gate kernels,
    branch choice on the host) makes the same choices, so <Z_q> agree to
    complex64 rounding; and every trajectory is the oracle's run with the
    same Philox draws."""
    batch = _traj_batch(24, 10, 14, 6, 1300, 0.08)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    zg, ig = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=55)
    zd, idr = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=55, direct_launch=True)
    zh, ih = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=55, plan=qs.PLAN_UNFUSED)
    assert ig["graph"] == 1 and idr["graph"] == 0 and ig["host_sampled"] == 0
    assert ig["passes"] >= 2 and ig["jumps"] > 0 and ig["jumps"] == idr["jumps"] == ih["jumps"]
    assert ih["passes"] == 0 and ih["host_sampled"] == len(batch)
    assert np.array_equal(zg, zd)
    assert np.max(np.abs(zg - zh)) <= 1e-4
    off = 0
    for t, (n, ops) in enumerate(batch):
        psi, _ = oracle.run(n, ops, seed=55, traj=t)
        assert np.max(np.abs(zg[off:off + n] - oracle.expect_z(psi))) <= 1e-4, (t, n)
        off += n


def test_trajectory_autotune_runs_every_width_set_exactly(qs):
    """QS_PLAN_AUTOTUNE: each of the first calls for a batch shape runs the
    next candidate width set (tile qubits, block width, outer bits) over the
    whole batch; every call is an exact run (the oracle's <Z_q> per
    trajectory), and once all are measured the fastest is kept.  A call that
    had to enlarge the job buffers kept between calls is not recorded (its
    candidate runs again), so a call adds at most one measured candidate."""
    batch = _traj_batch(8, 14, 15, 4, 1400, 0.05)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    want = np.concatenate([oracle.expect_z(oracle.run(n, ops, seed=57, traj=t)[0])
                           for t, (n, ops) in enumerate(batch)])
    seen = set()
    ncand, tried = None, 0
    for call in range(24):
        z, info = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=57, plan=qs.PLAN_AUTOTUNE)
        assert np.max(np.abs(z - want)) <= 1e-4, call
        ncand = info["autotune_candidates"]
        assert info["autotune_tried"] in (tried, tried + 1), call
        tried = info["autotune_tried"]
        seen.add((info["tile_qubits"], info["k_max"], info["max_outer"], info["chunk"]))
        if tried == ncand:
            break
    assert ncand >= 2 and tried == ncand and len(seen) == ncand


def test_batched_trajectories_wider_than_a_tile(qs):
    """States of 14..16 qubits span several 13-qubit tiles, so the batched
    sweeps select operators on the qubits outside the tile; each trajectory
    is still the oracle's run with the same draws."""
    batch = _traj_batch(6, 14, 16, 4, 900, 0.05)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    z, sec = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=33)
    off = 0
    for t, (n, ops) in enumerate(batch):
        psi, _ = oracle.run(n, ops, seed=33, traj=t)
        assert np.max(np.abs(z[off:off + n] - oracle.expect_z(psi))) <= 1e-4, (t, n)
        off += n


def test_trajectory_error_in_a_later_job_then_a_clean_batch(qs):
    """Trajectories are prepared job by job (at most 128 per job): a circuit
    with a qubit beyond its trajectory's width in the second job still fails
    the call with QS_E_RANGE, and the next call, on the job buffers kept
    from the failed one, matches the oracle."""
    batch = _traj_batch(6, 10, 11, 3, 920, 0.05)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    r, c = cg.grid_shape(12)
    bad = qs.Circuit(cg.random_circuit(r, c, 3, 921, dep1=0.05, dep2=0.05, damping=0.05))
    with pytest.raises(qs.QSError) as err:
        qs.run_trajectories(circs * 25 + [bad], widths * 25 + [10], dtype=qs.C64, seed=35)
    assert err.value.status == -2  # QS_E_RANGE
    z, _ = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=35)
    off = 0
    for t, (n, ops) in enumerate(batch):
        psi, _ = oracle.run(n, ops, seed=35, traj=t)
        assert np.max(np.abs(z[off:off + n] - oracle.expect_z(psi))) <= 1e-4, (t, n)
        off += n


@pytest.mark.parametrize("n,T,dtype", [(12, 3, "c64"), (28, 1, "c64"), (33, 1, "c64"),
                                       (12, 3, "c128"), (26, 1, "c128"), (33, 1, "c128")])
def test_batched_trajectories_product_state_closed_form(qs, n, T, dtype):
    """Ry(theta_q) on every qubit, then amplitude damping on every qubit in
    ascending order (one run of n damping sites): the state stays a product
    state, so each trajectory is n independent one-qubit Sec. 2.4 steps with
    the same Philox draws (site q is the q-th damping site), done here per
    qubit with the oracle's one-qubit noisy gate.  The widths reach every
    form of the run-sum kernel: runs of up to 24 or 36 sites, and at 33
    qubits (a 64 GiB complex64 or 128 GiB complex128 state) 64-bit group
    bits.  The batch run twice gives bit-identical results."""
    rng = np.random.default_rng(5150 + n)
    theta = rng.uniform(0.0, np.pi, n)
    gamma = rng.uniform(0.05, 0.6, n)
    ops = [cg.Gate((q,), (), cg.ry(theta[q])) for q in range(n)]
    for q in range(n):
        ops.append(cg.Gate((q,), (), np.eye(2, dtype=np.complex128), "id"))
        ops.append(cg.Noise((q,), cg.kraus_amplitude_damping(gamma[q]), "amplitude_damping"))
    c = qs.Circuit(ops)
    seed = 91
    dt = qs.C64 if dtype == "c64" else qs.C128
    tol = 1e-4 if dtype == "c64" else 1e-9
    z, _ = qs.run_trajectories([c] * T, [n] * T, dtype=dt, seed=seed)
    for t in range(T):
        want = np.empty(n)
        for q in range(n):
            psi = np.array([1.0, 0.0], dtype=np.complex128)
            oracle.apply_noisy(psi, [0], cg.ry(theta[q]), cg.kraus_amplitude_damping(gamma[q]),
                               oracle.uniform(seed, t, q))
            p0, p1 = abs(psi[0]) ** 2, abs(psi[1]) ** 2
            want[q] = (p0 - p1) / (p0 + p1)
        assert np.max(np.abs(z[t * n:(t + 1) * n] - want)) <= tol, t
    if n <= 16:
        z2, _ = qs.run_trajectories([c] * T, [n] * T, dtype=dt, seed=seed)
        assert np.array_equal(z, z2)


def test_batched_trajectory_mean_matches_density_matrix(qs):
    """Amplified rates (5e-2 everywhere), where a wrong branch weight or
    Kraus product moves the mean well beyond the sampling error."""
    n = 10
    ops = cg.random_circuit(2, 5, 6, seed=4010, dep1=0.05, dep2=0.05, damping=0.05)
    rho = oracle.dm_run(n, ops)
    zdm = oracle.dm_expect_z(rho)
    T = 4096
    c = qs.Circuit(ops)
    z, sec = qs.run_trajectories([c] * T, [n] * T, dtype=qs.C64, seed=77)
    zs = z.reshape(T, n)
    mean = zs.mean(axis=0)
    sigma = np.maximum(zs.std(axis=0), 1e-3)
    assert np.all(np.abs(mean - zdm) < 5 * sigma / math.sqrt(T)), (mean, zdm)


def test_batched_trajectory_mean_at_workload_rates(qs):
    """The trajectory workload's own rates (depolarizing 1e-3 / 1e-2, damping
    5e-4 per layer) on the 10-qubit depth-24 circuit: the mean of 4096
    trajectories against the stored exact density-matrix values."""
    n = 10
    ops = cg.random_circuit(2, 5, 24, seed=4010, dep1=1e-3, dep2=1e-2, damping=5e-4)
    zdm = np.loadtxt(os.path.join(GOLDEN, "dm_n10_d24_workload_rates.txt"))
    T = 4096
    z, sec = qs.run_trajectories([qs.Circuit(ops)] * T, [n] * T, dtype=qs.C64, seed=78)
    zs = z.reshape(T, n)
    sigma = np.maximum(zs.std(axis=0), 1e-3)
    assert np.all(np.abs(zs.mean(axis=0) - zdm) < 5 * sigma / math.sqrt(T)), (zs.mean(axis=0), zdm)


# ---------------------------------------------------------------- autotune --


@pytest.mark.parametrize("dtype,ncand", [("c64", 6), ("c128", 3)])
def test_autotune_runs_every_candidate_exactly(qs, dtype, ncand):
    """Each autotuning run executes one candidate plan completely; every run,
    and the tuned runs after it, agree with the oracle."""
    rows, cols = (4, 5) if dtype == "c64" else (3, 5)
    n = rows * cols
    ops = cg.random_circuit(rows, cols, 16, seed=321, cu3_prob=0.1)
    ref, _ = oracle.run(n, ops)
    dt = qs.C64 if dtype == "c64" else qs.C128
    c = qs.Circuit(ops)
    s = qs.State(n, dt)
    for r in range(ncand + 2):
        s.reset()
        s.run(c, plan=qs.PLAN_AUTOTUNE)
        got = s.amplitudes()
        if dtype == "c64":
            assert infidelity(ref, got) <= 1e-6, r
        else:
            assert np.max(np.abs(got - ref)) <= TOL128, r
        tried, cands, tq, km, sec = c.autotune_result(n, dt)
        assert cands == ncand and tried == min(r + 1, ncand)
        assert sec > 0
    assert (tq in (11, 12, 13) and km in (4, 5)) if dtype == "c64" else (tq == 0 and km in (2, 3, 4))
    s.close()


# --------------------------------------------------------------- cost model --


def test_mlp_forward_and_gradient_match_fp64_oracle(qs):
    rng = np.random.default_rng(3)
    f = qs.COST_FEATURES
    p = (rng.standard_normal(qs.mlp_num_params(f)) * 0.3).astype(np.float32)
    x = rng.standard_normal((300, f)).astype(np.float32)
    t = rng.standard_normal(300).astype(np.float32)
    y = qs.mlp_forward(p, x)
    yr, lossr, gr = oracle.mlp_forward_backward(p.astype(np.float64), f, 64, x.astype(np.float64),
                                                t.astype(np.float64))
    assert np.max(np.abs(y - yr)) <= 1e-4 * max(1.0, np.max(np.abs(yr)))
    loss, g = qs.mlp_grad(p, x, t)
    assert abs(loss - lossr) <= 1e-4 * max(1.0, lossr)
    assert np.max(np.abs(g - gr)) <= 1e-4 * max(1.0, np.max(np.abs(gr)))


def test_mlp_training_reduces_loss(qs):
    rng = np.random.default_rng(5)
    f = qs.COST_FEATURES
    x = rng.uniform(0, 1, (2048, f)).astype(np.float32)
    t = (np.sin(3 * x[:, 0]) + x[:, 1] * x[:, 2] - 0.5 * x[:, 3]).astype(np.float32)
    p0 = qs.mlp_init(1)
    _, l0, _ = oracle.mlp_forward_backward(p0.astype(np.float64), f, 64, x.astype(np.float64),
                                           t.astype(np.float64))
    p1, _ = qs.mlp_train(p0, x, t, steps=1500, batch=256, lr=3e-3, seed=2)
    _, l1, _ = oracle.mlp_forward_backward(p1.astype(np.float64), f, 64, x.astype(np.float64),
                                           t.astype(np.float64))
    assert l1 < 0.05 * l0, (l0, l1)


@pytest.fixture(scope="module")
def cost_model(qs):
    """The planner's cost network trained on the simulator's own timings:
    profiled tile sweeps of random circuits under every tile shape; 20% of
    the samples are held out."""
    n = 24
    s = qs.State(n, qs.C64)
    s.profile(True)
    for i in range(8):
        rows, cols = [(4, 6), (6, 4), (3, 8), (8, 3)][i % 4]
        c = qs.Circuit(cg.random_circuit(rows, cols, 12, seed=9000 + i, cu3_prob=0.1))
        for m in (11, 12, 13):
            for k in (4, 5):
                s.reset()
                s.run(c, plan=qs.PLAN_GREEDY, k_max=k, tile_qubits=m)
    X, y = s.profile_samples()
    s.profile(False)
    s.close()
    rng = np.random.default_rng(0)
    perm = rng.permutation(X.shape[0])
    tr, te = perm[: int(0.8 * len(perm))], perm[int(0.8 * len(perm)):]
    p, _ = qs.mlp_train(qs.mlp_init(4), X[tr], y[tr], steps=3000, batch=256, lr=2e-3, seed=7)
    return p, X[te], y[te], X.shape[0]


def test_cost_model_predicts_held_out_sweeps_and_learned_plans_are_exact(qs, cost_model):
    """The trained network predicts held-out sweep times (correlation > 0.8),
    and plans it chooses apply the circuit exactly (oracle, 16 and 20
    qubits)."""
    p, Xte, yte, nsamp = cost_model
    assert nsamp > 200
    corr = np.corrcoef(qs.mlp_forward(p, Xte), yte)[0, 1]
    assert corr > 0.8, corr
    qs.cost_model_set(p)
    try:
        for rows, cols, depth in [(4, 4, 20), (4, 5, 24)]:
            ops = cg.random_circuit(rows, cols, depth, seed=77, cu3_prob=0.1)
            ref, _ = oracle.run(rows * cols, ops)
            t = qs.State(rows * cols, qs.C64)
            t.run(qs.Circuit(ops), plan=qs.PLAN_LEARNED)
            assert infidelity(ref, t.amplitudes()) <= 1e-6
            t.close()
    finally:
        qs.cost_model_set(None)


def test_learned_planner_measured_ratio_on_held_out_circuits(qs, cost_model):
    """What the trained network gains over the plan without it, measured:
    three held-out 24-qubit circuits, each plan warmed up past its
    tile-order timing runs (QS_TILE_ORDERS + 1 runs), then the median of
    five timed runs.  The ratio greedy / learned is printed per circuit
    ("no gain" when the network keeps the greedy plan or does not beat
    it).  The learned plan is the greedy plan unless the network predicts
    it at least 3% cheaper, so a large loss would mean the network is
    wrong about whole plans: the geometric mean must stay above 0.9."""
    import time
    p = cost_model[0]
    n = 24
    s = qs.State(n, qs.C64)
    ratios = []
    try:
        for seed, (rows, cols) in zip((9991, 9992, 9993), ((4, 6), (6, 4), (3, 8))):
            held = qs.Circuit(cg.random_circuit(rows, cols, 24, seed=seed, cu3_prob=0.1))
            times = {}
            for plan in (qs.PLAN_GREEDY, qs.PLAN_LEARNED):
                qs.cost_model_set(p if plan == qs.PLAN_LEARNED else None)
                for _ in range(qs.TILE_ORDERS + 1):
                    s.reset()
                    s.run(held, plan=plan)
                runs = []
                for _ in range(5):
                    s.reset()
                    s.synchronize()
                    t0 = time.perf_counter()
                    s.run(held, plan=plan)
                    s.synchronize()
                    runs.append(time.perf_counter() - t0)
                times[plan] = float(np.median(runs))
            qs.cost_model_set(p)
            same = held.plan_info(n, qs.C64, qs.PLAN_LEARNED) == held.plan_info(n, qs.C64, qs.PLAN_GREEDY)
            r = times[qs.PLAN_GREEDY] / times[qs.PLAN_LEARNED]
            ratios.append(r)
            print("held-out %dx%d: greedy %.4f s, learned %.4f s, greedy/learned %.3f%s"
                  % (rows, cols, times[qs.PLAN_GREEDY], times[qs.PLAN_LEARNED], r,
                     " (same plan: no gain)" if same else ("" if r > 1.0 else " (no gain)")), flush=True)
    finally:
        qs.cost_model_set(None)
        s.close()
    gm = float(np.exp(np.mean(np.log(ratios))))
    print("geometric mean greedy/learned %.3f" % gm, flush=True)
    assert gm > 0.9


# ------------------------------------------------ sharded states: remap --


def _remap_index(b, L, lq):
    """Shard index of element b of a packed remap buffer, as qs.h documents it:
    the chunk number b >> (L - g) spread over the qubits lq (bit i at lq[i]),
    the rest of b over the other local qubits in ascending order."""
    g = len(lq)
    d, x = b >> (L - g), b & ((1 << (L - g)) - 1)
    idx = 0
    for k, p in enumerate(p for p in range(L) if p not in lq):
        idx |= ((x >> k) & 1) << p
    for i, q in enumerate(lq):
        idx |= ((d >> i) & 1) << q
    return idx


class _StateBuffer:
    """Device memory for a remap buffer: the amplitude array of another state
    (its initialisation finished before use), readable and writable through
    that state's own calls."""

    def __init__(self, qs, L, dt):
        self.s = qs.State(L, dt)
        self.s.synchronize()

    def data_ptr(self):
        return self.s.info()["device_ptr"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,lq", [(9, []), (8, [3]), (10, [7, 0]), (12, [5, 1, 11]),
                                  (11, [0, 1, 2]), (12, [11, 10, 9]), (6, [5, 0, 3, 1, 4, 2])])
def test_remap_exchange_swaps_global_and_local_qubits(qs, dtype, L, lq):
    """An (L + g)-qubit state split into 2^g shards of L qubits (one per
    would-be device, all on this one): each packed buffer holds the layout
    qs.h documents; after the all-to-all (chunk d of shard r to slot r of
    shard d, done on the host here) and the unpacks, the shards equal the
    oracle's state after SWAP(L + i, lq[i]) for every i, bit for bit (data
    movement only)."""
    g, n = len(lq), L + len(lq)
    dt = qs.C128 if dtype == "c128" else qs.C64
    psi = cg.random_state(n, 7000 + 31 * L + g)
    if dt == qs.C64:
        psi = psi.astype(np.complex64).astype(np.complex128)
    ref = psi.copy()
    for i, q in enumerate(lq):
        oracle.apply(ref, (L + i, q), (), oracle.named_gate("SWAP"))
    size, chunk = 1 << L, 1 << (L - g)
    shards, sent = [], []
    for r in range(1 << g):
        s = qs.State(L, dt)
        s.set_amplitudes(psi[r * size:(r + 1) * size])
        b = _StateBuffer(qs, L, dt)
        s.remap_pack(lq, b)
        s.synchronize()
        sent.append(b.s.amplitudes())
        b.s.close()
        shards.append(s)
    layout = np.array([_remap_index(b, L, lq) for b in range(size)])
    for r in range(1 << g):
        assert np.array_equal(sent[r], psi[r * size + layout])
    for d, s in enumerate(shards):
        recv = np.concatenate([sent[r][d * chunk:(d + 1) * chunk] for r in range(1 << g)])
        b = _StateBuffer(qs, L, dt)
        b.s.set_amplitudes(recv)
        s.remap_unpack(lq, b)
        s.synchronize()
        b.s.close()
    got = np.concatenate([s.amplitudes() for s in shards])
    assert np.array_equal(got, ref)
    for s in shards:
        s.close()


@pytest.mark.parametrize("dtype,L,lq", [("c64", 27, [4, 17, 26]), ("c64", 26, [0, 25, 12]),
                                        ("c128", 26, [9, 3, 25, 14])])
def test_remap_large_shard_sampled_chunks_and_round_trip(qs, dtype, L, lq):
    """At shard sizes of 0.5-1 GiB, on a state prepared by two layers of
    random one-qubit gates with a CZ layer between them: 2^16 sampled entries
    of the packed buffer equal the shard amplitudes the documented layout
    names, and unpacking the buffer into a reset shard restores those
    amplitudes exactly and the FP64 norm."""
    dt = qs.C128 if dtype == "c128" else qs.C64
    rng = np.random.default_rng(9000 + L)
    s = qs.State(L, dt)
    for q in range(L):
        s.apply_gate((q,), (), cg.random_unitary(2, rng))
    for q in range(0, L - 1, 2):
        s.apply_gate((q, q + 1), (), np.diag([1, 1, 1, -1]))
    for q in range(L):
        s.apply_gate((q,), (), cg.random_unitary(2, rng))
    bs = np.sort(rng.choice(1 << L, size=1 << 16, replace=False)).astype(np.uint64)
    src = np.array([_remap_index(int(b), L, lq) for b in bs], dtype=np.uint64)
    before = s.amplitudes(src)
    norm_before = s.norm()
    buf = _StateBuffer(qs, L, dt)
    s.remap_pack(lq, buf)
    s.synchronize()
    assert np.array_equal(buf.s.amplitudes(bs), before)
    s.reset()
    s.remap_unpack(lq, buf)
    assert np.array_equal(s.amplitudes(src), before)
    assert abs(s.norm() - norm_before) < 1e-12
    buf.s.close()
    s.close()


def test_remap_validation(qs):
    s = qs.State(6, qs.C128)
    buf = _StateBuffer(qs, 6, qs.C128)
    for lq, status in [([6], -2), ([1, 1], -2), ([-1], -2), (list(range(7)), -1)]:
        with pytest.raises(qs.QSError) as e:
            s.remap_pack(lq, buf)
        assert e.value.status == status

    class Ptr:
        def __init__(self, p):
            self.p = p

        def data_ptr(self):
            return self.p

    with pytest.raises(qs.QSError) as e:
        s.remap_unpack([0], Ptr(buf.data_ptr() + 8))
    assert e.value.status == -1 and "aligned" in qs.last_error()
    with pytest.raises(qs.QSError) as e:
        s.remap_pack([0], Ptr(0))
    assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        s.remap_pack([0], Ptr(s.info()["device_ptr"] + 128))
    assert e.value.status == -1 and "overlaps" in qs.last_error()
    big = qs.State(12, qs.C64)
    with pytest.raises(qs.QSError) as e:
        big.remap_pack(list(range(11)), Ptr(buf.data_ptr()))
    assert e.value.status == -1
    for x in (s, big, buf.s):
        x.close()


# ------------------------------------------------ partial-amplitude mode --


def _partial_circuit():
    """12 qubits (4 x 3 grid, depth 4: the CZ layer 3 crosses rows 1 | 2 with
    3 gates) plus one crossing gate of every supported form: CNOT both ways,
    CR, Toffoli with both controls across, CU3, a 3-qubit diagonal with one
    qubit in part A, and a CONTROL group from part A around a part-B gate."""
    rng = np.random.default_rng(77)
    ops = list(cg.random_circuit(4, 3, 4, seed=7001, cu3_prob=0.0))
    d3 = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 8)))
    cr = np.diag([1, np.exp(0.7j)])
    extra = [cg.Gate((7,), (1,), cg.PX), cg.Gate((2,), (8,), cg.PX), cg.Gate((9,), (3,), cr),
             cg.Gate((10,), (0, 4), cg.PX), cg.Gate((0,), (11,), cg.u3(0.4, 1.1, -0.3)),
             cg.Gate((5, 6, 11), (), d3), cg.Marker("control", 2), cg.Gate((8,), (), cg.H_GATE),
             cg.Marker("endcontrol")]
    return ops[:20] + extra[:3] + ops[20:40] + extra[3:] + ops[40:]


@pytest.mark.parametrize("dtype,plan", [("c128", "unfused"), ("c128", "greedy"), ("c64", "unfused"),
                                        ("c64", "greedy")])
def test_partial_amplitudes_match_oracle_full_state(qs, dtype, plan):
    """Partial-amplitude mode (Sec. 2.2 (partial), Eq. 4): every amplitude of a
    12-qubit circuit cut between qubits 0-5 and 6-11 (10 cuts, 1024 branch
    words, 2048 six-qubit sub-circuits) equals the oracle's full-amplitude
    state: complex128 within 1e-12, complex64 within infidelity 1e-6."""
    ops = _partial_circuit()
    n, part_a = 12, (1 << 6) - 1
    ref, _ = oracle.run(n, ops)
    c = qs.Circuit(ops)
    dt = qs.C128 if dtype == "c128" else qs.C64
    pl = qs.PLAN_UNFUSED if plan == "unfused" else qs.PLAN_GREEDY
    got, cuts = c.partial_amplitudes(n, part_a, np.arange(1 << n), dtype=dt, plan=pl)
    assert cuts == 10 == c.partial_cuts(n, part_a)
    if dt == qs.C128:
        assert np.max(np.abs(got - ref)) <= TOL128
    else:
        assert infidelity(ref, got) <= 1e-6
        assert np.max(np.abs(got - ref)) <= 2e-5


def test_partial_amplitudes_other_division_and_sampled_order(qs):
    """The same circuit divided into an interleaved part A (even qubits):
    CZ layers, CU3 and every extra gate cross differently; amplitudes asked in
    a shuffled order with repeats come back in that order (complex128)."""
    ops = _partial_circuit()[:30]
    n, part_a = 12, 0b010101010101
    ref, _ = oracle.run(n, ops)
    c = qs.Circuit(ops)
    cuts = c.partial_cuts(n, part_a)
    assert 1 <= cuts <= 14
    idx = np.random.default_rng(5).integers(0, 1 << n, size=3000)
    got, cc = c.partial_amplitudes(n, part_a, idx)
    assert cc == cuts
    assert np.max(np.abs(got - ref[idx])) <= TOL128


def test_partial_amplitudes_per_branch_path_matches_tree_walk(qs):
    """With a memory limit below the c + 1 states per part that the
    depth-first walk keeps, every branch word runs its sub-circuits in full;
    both ways give the oracle's amplitudes (complex128)."""
    ops = _partial_circuit()
    n, part_a = 12, (1 << 6) - 1
    ref, _ = oracle.run(n, ops)
    c = qs.Circuit(ops)
    qs.set_memory_limit(4 << 10)  # 2 x 64 x 16 B per level fit, 11 levels do not
    try:
        got, cuts = c.partial_amplitudes(n, part_a, np.arange(1 << n))
    finally:
        qs.set_memory_limit(0)
    assert cuts == 10
    assert np.max(np.abs(got - ref)) <= TOL128


def test_partial_amplitudes_30_qubits_against_full_state(qs):
    """At 30 qubits (6 x 5 grid, depth 8, divided between rows 2 and 3: 10
    cuts, two 15-qubit parts), 4096 sampled amplitudes equal those of the
    complex128 full-amplitude path (which the tests above pin to the oracle);
    with complex64 tiled sub-circuits, to the complex64 bar."""
    n, part_a = 30, (1 << 15) - 1
    ops = cg.random_circuit(6, 5, 8, seed=7002)
    c = qs.Circuit(ops)
    s = qs.State(n, qs.C128)
    s.run(c)
    idx = np.random.default_rng(6).choice(1 << n, size=4096, replace=False)
    full = s.amplitudes(idx)
    s.close()
    got, cuts = c.partial_amplitudes(n, part_a, idx)
    assert cuts == 10
    assert np.max(np.abs(got - full)) <= 1e-13
    # complex64 sub-circuits of 15 qubits run as tile sweeps
    got64, _ = c.partial_amplitudes(n, part_a, idx, dtype=qs.C64, plan=qs.PLAN_GREEDY)
    _check_c64_sample(got64, full)


def test_partial_amplitudes_40_qubits_two_divisions_agree(qs):
    """At 40 qubits (8 x 5 grid, depth 6), where no full state fits one GPU,
    two dividing lines give entirely different sub-circuits: rows 0-3 | 4-7
    (20 + 20 qubits, 5 cuts) and columns 0-1 | 2-4 (16 + 24 qubits, 8 cuts).
    Their amplitudes at 4096 sampled indices agree to 1e-13 (complex128), and
    the mean of |amp|^2 * 2^40 over the sample is near 1."""
    rows, cols, n = 8, 5, 40
    ops = cg.random_circuit(rows, cols, 6, seed=6003)
    c = qs.Circuit(ops)
    top = (1 << 20) - 1
    left = sum(1 << (r * cols + k) for r in range(rows) for k in range(2))
    idx = np.random.default_rng(8).integers(0, 1 << n, size=4096, dtype=np.uint64)
    a, ca = c.partial_amplitudes(n, top, idx, plan=qs.PLAN_GREEDY)
    b, cb = c.partial_amplitudes(n, left, idx, plan=qs.PLAN_GREEDY)
    assert (ca, cb) == (5, 8)
    assert np.max(np.abs(a - b)) <= 1e-13
    assert abs(np.mean(np.abs(a) ** 2) * 2.0 ** n - 1) < 0.25


def test_partial_amplitudes_validation(qs):
    c = qs.Circuit([cg.Gate((0,), (), cg.H_GATE), cg.Gate((0, 5), (), cg.CZ_GATE)])
    with pytest.raises(qs.QSError) as e:
        c.partial_amplitudes(6, 0b111, [64])
    assert e.value.status == -2
    with pytest.raises(qs.QSError) as e:
        c.partial_amplitudes(6, 0b111, [1], plan=qs.PLAN_AUTOTUNE)
    assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        c.partial_amplitudes(6, 0b111, [1], dtype=9)
    assert e.value.status == -1
    got, cuts = c.partial_amplitudes(6, 0b111, [])
    assert got.size == 0 and cuts == 1


# --------------------------------------------------------------- scripts --


def test_script_run_reproduces_the_printed_appA2_output(qs):
    """The App. A-2 example through the library's own script reader: the
    PMEASURE probabilities equal the printed output within 1e-6 and the
    oracle's (run on the test-side reading of the same script) within 1e-12."""
    with open(os.path.join(GOLDEN, "appA2_example.txt")) as f:
        full = f.read()
    n, ops, pm, printed = appa_script.parse(full, oracle.named_gate)
    ref, _ = oracle.run(n, ops)
    want = oracle.probabilities(ref, pm)
    creg, probs, info = qs.script_run(full.split("%Output")[0])
    assert info["pmeasure"] == pm and creg == [0, 0, 0]
    assert np.max(np.abs(probs - printed)) <= 1e-6
    assert np.max(np.abs(probs - want)) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_script_gate_table_matches_oracle(qs, dtype):
    """Every App. A-1 instruction (angle expressions, nested DAGGER and
    CONTROL groups) parsed by the library and run on a state gives the
    oracle's amplitudes for the test-side reading with the oracle's gate
    table."""
    from tests.test_abi_host import SCRIPT_ALL
    n, ops, _, _ = appa_script.parse(SCRIPT_ALL, oracle.named_gate)
    ref, _ = oracle.run(n, ops)
    c, info = qs.script_parse(SCRIPT_ALL)
    dt = qs.C128 if dtype == "c128" else qs.C64
    s = qs.State(n, dt)
    s.run(c)
    got = s.amplitudes()
    s.close()
    tol = TOL128 if dt == qs.C128 else 1e-6
    assert np.max(np.abs(got - ref)) <= tol


def _measure_ops(qubits):
    p0, p1 = np.diag([1.0, 0.0]).astype(complex), np.diag([0.0, 1.0]).astype(complex)
    out = []
    for q in qubits:
        out += [cg.Gate((q,), (), np.eye(2)), cg.Noise((q,), np.stack([p0, p1]))]
    return out


def test_script_measure_outcomes_match_oracle_draws(qs):
    """MEASURE i, $j is the Sec. 2.4 noise site with Kraus {P0, P1}: over 24
    seeds the outcomes equal the oracle's branch choices for the same Philox
    draws, a Bell pair measures equal bits, an X-flipped qubit measures 1,
    and a measured qubit stays collapsed (PMEASURE is then one-hot)."""
    script = "QINIT 4\nCREG 4\nH 0\nCNOT 0, 1\nX 2\nRY 3, \"1.1\"\nMEASURE 0, $0\nMEASURE 1, $1\n" \
             "MEASURE 2, $2\nMEASURE 3, $3\nPMEASURE 3\n"
    ops = [cg.Gate((0,), (), oracle.named_gate("H")), cg.Gate((1,), (0,), oracle.named_gate("X")),
           cg.Gate((2,), (), oracle.named_gate("X")), cg.Gate((3,), (), oracle.named_gate("RY", (1.1,)))]
    ops += _measure_ops([0, 1, 2, 3])
    seen = set()
    for seed in range(24):
        creg, probs, info = qs.script_run(script, seed=seed)
        _, chosen = oracle.run(4, ops, seed=seed)
        assert creg == list(chosen), seed
        assert creg[0] == creg[1] and creg[2] == 1
        assert probs[creg[3]] == pytest.approx(1.0, abs=1e-12) and info["measures"] == 4
        seen.add(creg[0])
    assert seen == {0, 1}


# ------------------------------------------------ single-amplitude mode --


def _bitstrings(n, count, seed, extra=()):
    rng = np.random.default_rng(seed)
    b = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.concatenate([np.array(list(extra), dtype=np.uint64), b])


@pytest.mark.parametrize("rows,cols,depth,nslice", [(3, 4, 10, 0), (4, 4, 12, 0), (4, 4, 12, 3), (4, 5, 8, 5)])
def test_single_amplitudes_match_oracle(qs, rows, cols, depth, nslice):
    """Sec. 2.3: <x|C|0...0> from the graphical model's eliminations equals
    the oracle's full-amplitude entry x (complex128 bound 1e-12), with and
    without slicing (2^nslice graphs summed)."""
    n = rows * cols
    ops = cg.random_circuit(rows, cols, depth, seed=1500 + n + depth, cu3_prob=0.1)
    ref, _ = oracle.run(n, ops)
    bits = _bitstrings(n, 64, n + nslice, [0, (1 << n) - 1, 1, 1 << (n - 1)])
    print("[single] n=%d depth=%d nslice=%d" % (n, depth, nslice), flush=True)
    got, info = qs.Circuit(ops).single_amplitudes(n, bits, nslice)
    assert info["sliced"] == nslice and info["batch"] >= (1 << nslice)
    assert np.max(np.abs(got - ref[bits.astype(np.int64)])) <= TOL128


def test_single_amplitudes_every_gate_form_groups_and_idle_qubit(qs):
    """Dense gates of 1-6 targets with controls, diagonal gates of up to four
    qubits, DAGGER and CONTROL groups, and a qubit no gate touches (its
    amplitudes with bit 9 set are exactly 0): all 1024 amplitudes of a
    10-qubit circuit against the oracle's state."""
    n = 10
    ops = _mixed_circuit(9, 40, 1601)
    full = ([cg.Marker("control", 8)] + list(ops[:12]) + [cg.Marker("endcontrol")]
            + [cg.Marker("dagger")] + list(ops[12:30]) + [cg.Marker("enddagger")] + list(ops[30:])
            + [cg.Gate((3,), (), cg.T_GATE), cg.Gate((0, 5), (), cg.CZ_GATE)])
    ref, _ = oracle.run(n, full)
    bits = np.arange(1 << n, dtype=np.uint64)
    got, info = qs.Circuit(full).single_amplitudes(n, bits, 2)
    assert np.max(np.abs(got - ref)) <= TOL128
    assert np.all(got[512:] == 0)


@pytest.mark.parametrize("parts", [2, 3])
def test_single_amplitudes_wide_product_circuits(qs, parts):
    """40 and 60 qubits (no full state fits anywhere): `parts` independent
    20-qubit depth-8 random circuits on the qubits q with q mod parts = j,
    interleaved gate by gate.  The graph falls apart into `parts`
    components and every amplitude is the product of the oracle's
    amplitudes of the parts."""
    nh = 20
    n = parts * nh
    halves = [cg.random_circuit(4, 5, 8, seed=1700 + j, cu3_prob=0.1) for j in range(parts)]
    placed = []
    for j, h in enumerate(halves):
        placed.append([cg.Gate(tuple(parts * q + j for q in o.targets),
                               tuple(parts * q + j for q in o.controls), o.matrix, o.name) for o in h])
    ops = [g for group in zip(*placed) for g in group]
    refs = [oracle.run(nh, h)[0] for h in halves]
    bits = _bitstrings(n, 48, 1750 + parts, [0, (1 << n) - 1, 1 << (n - 1)])
    want = np.ones(bits.size, dtype=np.complex128)
    for j in range(parts):
        sub = np.zeros(bits.size, dtype=np.int64)
        for b in range(nh):
            sub |= ((bits >> np.uint64(parts * b + j)) & np.uint64(1)).astype(np.int64) << b
        want *= refs[j][sub]
    print("[single] %d qubits, %d parts" % (n, parts), flush=True)
    got, info = qs.Circuit(ops).single_amplitudes(n, bits)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-10 * scale


def test_single_amplitudes_36_qubit_product_with_both_operand_layouts(qs):
    """A 36-qubit circuit of two independent 18-qubit depth-10 circuits on
    the even and odd qubits: its merges store some operands with their own
    vertices lowest and the others with the summed vertices lowest (both
    forms are read by every merge kernel); the amplitudes are products of
    the oracle's 18-qubit amplitudes."""
    nh = 18
    half = cg.random_circuit(3, 6, 10, seed=1901, cu3_prob=0.1)
    half2 = cg.random_circuit(6, 3, 10, seed=1902, cu3_prob=0.1)
    ops = _product_circuit(half, half2, nh)
    bits = _bitstrings(2 * nh, 40, 1903, [0, (1 << 36) - 1])
    want = _product_expected(half, half2, nh, bits)
    c = qs.Circuit(ops)
    info = c.single_plan(2 * nh)
    assert info["own_low"] > 0 and info["own_low"] < info["tensors"]
    got, _ = c.single_amplitudes(2 * nh, bits)
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_single_amplitudes_in_bitstring_chunks(qs):
    """A memory bound smaller than the tensors of every bitstring at once
    makes the call process the bitstrings in chunks: the results are the
    same as in one chunk and the oracle's."""
    rows, cols, depth = 4, 4, 10
    n = rows * cols
    ops = cg.random_circuit(rows, cols, depth, seed=1801, cu3_prob=0.1)
    ref, _ = oracle.run(n, ops)
    bits = _bitstrings(n, 300, 1802)
    c = qs.Circuit(ops)
    one, i1 = c.single_amplitudes(n, bits, 1)
    peak = c.single_plan(n, 1)["peak_bytes"]
    qs.set_memory_limit(int(peak * 7))
    try:
        chunked, i2 = c.single_amplitudes(n, bits, 1)
    finally:
        qs.set_memory_limit(0)
    assert i2["batch"] < i1["batch"]
    assert np.max(np.abs(one - ref[bits.astype(np.int64)])) <= TOL128
    assert np.max(np.abs(chunked - one)) <= 1e-15
