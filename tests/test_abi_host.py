"""Host-side checks of the C ABI: the library loads, exports every symbol
include/qs.h declares, and validates arguments before touching a device.
No call here reaches the GPU."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2008_07140_amd import circuits as cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def qs():
    lib = os.path.join(ROOT, "paper_2008_07140_amd", "libqs.so")
    if not os.path.exists(lib):
        from paper_2008_07140_amd import build
        build.build(verbose=False)
    from paper_2008_07140_amd import qs as mod
    return mod


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "qs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_all_exported(qs):
    syms = declared_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(qs.lib(), s), s
    # the binding wraps exactly the declared calls
    assert sorted(qs.EXPORTED) == syms


def test_philox_known_answers_and_agreement_with_oracle(qs):
    assert qs.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert qs.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                            [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                          0x24126EA1]
    rng = np.random.default_rng(1)
    for _ in range(200):
        seed, traj, site = (int(x) for x in rng.integers(0, 2**63, size=3))
        assert qs.philox_uniform(seed, traj, site) == oracle.uniform(seed, traj, site)


def test_create_validation_without_device(qs):
    with pytest.raises(qs.QSError) as e:
        qs.State(0)
    assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        qs.State(3, dtype=7)
    assert e.value.status == -1
    qs.set_memory_limit(1 << 20)
    try:
        with pytest.raises(qs.QSError) as e:
            qs.State(20, qs.C128)  # 16 MiB > 1 MiB
        assert e.value.status == -3
        assert "memory limit" in qs.last_error()
    finally:
        qs.set_memory_limit(0)


def test_remap_rejects_a_missing_state(qs):
    lib = qs.lib()
    assert lib.qs_remap_pack(None, 0, None, None) == -1
    assert lib.qs_remap_unpack(None, 0, None, None) == -1
    assert "state is NULL" in qs.last_error()


def test_circuit_validation(qs):
    c = qs.Circuit()
    with pytest.raises(qs.QSError) as e:
        c.append(cg.Gate((1, 1), (), np.eye(4)))
    assert e.value.status == -2
    with pytest.raises(qs.QSError) as e:
        c.append(cg.Gate((0,), (0,), np.eye(2)))
    assert e.value.status == -2
    with pytest.raises(qs.QSError) as e:
        c.append(cg.Gate((0,), (), np.array([[np.nan, 0], [0, 1]])))
    assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        c.append(cg.Gate(tuple(range(7)), (), np.eye(128)))
    assert e.value.status == -1
    # noise must follow a gate on the same targets
    with pytest.raises(qs.QSError):
        c.append(cg.Noise((0,), cg.kraus_depolarizing(0.1)))
    c.append(cg.Gate((0,), (), cg.H_GATE))
    with pytest.raises(qs.QSError):
        c.append(cg.Noise((1,), cg.kraus_depolarizing(0.1)))
    bad = cg.kraus_depolarizing(0.1).copy()
    bad[0] *= 1.01
    with pytest.raises(qs.QSError) as e:
        c.append(cg.Noise((0,), bad))
    assert "not complete" in qs.last_error()
    c.append(cg.Noise((0,), cg.kraus_depolarizing(0.1)))
    assert c.counts() == (1, 1, 1)


def test_circuit_group_expansion_counts(qs):
    ops = [cg.Gate((0,), (), cg.H_GATE), cg.Marker("control", 2), cg.Marker("dagger"),
           cg.Gate((0,), (), cg.T_GATE), cg.Gate((1,), (), np.eye(2)), cg.Marker("enddagger"),
           cg.Marker("endcontrol")]
    c = qs.Circuit(ops)
    assert c.counts() == (3, 0, 2)
    c2 = qs.Circuit([cg.Marker("dagger"), cg.Gate((0,), (), cg.H_GATE)])
    with pytest.raises(qs.QSError) as e:
        c2.counts()
    assert e.value.status == -1
    c3 = qs.Circuit([cg.Marker("control", 0), cg.Gate((1,), (), cg.H_GATE),
                     cg.Marker("enddagger")])
    with pytest.raises(qs.QSError):
        c3.counts()
    c4 = qs.Circuit([cg.Marker("control", 0), cg.Gate((0,), (), cg.H_GATE),
                     cg.Marker("endcontrol")])
    with pytest.raises(qs.QSError):
        c4.counts()


def test_workload_shapes():
    """The generator reproduces the CZ counts per pattern of the grids."""
    assert [len(cg.cz_pairs(4, 4, p)) for p in range(4)] == [8, 8, 4, 4]
    assert [len(cg.cz_pairs(6, 5, p)) for p in range(4)] == [12, 15, 12, 10]
    assert [len(cg.cz_pairs(8, 4, p)) for p in range(4)] == [16, 16, 8, 12]
    assert [len(cg.cz_pairs(17, 2, p)) for p in range(4)] == [17, 16, 0, 16]
    n, ops = cg.workload("rqc30_d40")
    assert n == 30 and cg.count_gates(ops) == 1200 + 490
    ncu3 = sum(1 for o in ops if o.name == "cu3")
    assert 80 < ncu3 < 160
    for o in ops:
        if o.kind == "gate":
            m = o.matrix
            assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-14)


def test_cost_model_validation(qs):
    import ctypes
    p = qs.mlp_init(0)
    ptr = p.ctypes.data_as(ctypes.c_void_p)
    with pytest.raises(qs.QSError) as e:
        qs._check(qs.lib().qs_cost_model_set(ptr, 7, 64))
    assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        qs._check(qs.lib().qs_cost_model_set(ptr, 16, 32))
    assert e.value.status == -6
    qs.cost_model_set(p)
    qs.cost_model_set(None)
    assert p.size == qs.mlp_num_params(16) == oracle.mlp_num_params(16, 64)


def test_tile_planner_terminates_on_wide_diagonals(qs):
    """Diagonal gates too wide for a tile op (more than k_max qubits inside
    the tile, or more outer qubits than an op may select on) go on their own
    instead of stalling the sweep planner."""
    rng = np.random.default_rng(8)
    d6 = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 64)))
    for qubits in [(0, 1, 2, 3, 4, 5), (14, 15, 16, 17, 18, 19), (2, 9, 14, 15, 18, 19)]:
        ops = [cg.Gate(qubits, (), d6), cg.Gate((0,), (), cg.H_GATE), cg.Gate(qubits[::-1], (), d6)]
        for m, k in [(13, 5), (10, 4)]:
            info = qs.Circuit(ops).plan_info(20, qs.C64, qs.PLAN_GREEDY, k_max=k, tile_qubits=m)
            assert info["gates"] == 3 and 1 <= info["sweeps"] <= 3


def test_tile_planner_sweep_counts_on_workload_circuits(qs):
    """The greedy tile planner with its search over tile qubits (local search
    from the first-come set and from seeded random sets, two-sweep lookahead,
    the cheaper of the plans with 16 and 32 restarts): on the 30-qubit
    depth-40 workload circuit it needs 28 sweeps of 13-qubit tiles (41 with
    first-come tile qubits), on the 34-qubit one 13 (20) with 88 blocks, and
    every logical gate is planned.  A regression guard on the planner's
    quality, not a parity check."""
    n, ops = cg.workload("rqc30_d40")
    info = qs.Circuit(ops).plan_info(n, qs.C64, qs.PLAN_GREEDY)
    assert info["gates"] == cg.count_gates(ops)
    assert info["sweeps"] <= 29
    assert info["blocks"] <= 200
    n, ops = cg.workload("rqc34_d24")
    info = qs.Circuit(ops).plan_info(n, qs.C64, qs.PLAN_GREEDY)
    assert info["gates"] == cg.count_gates(ops) and info["sweeps"] <= 13 and info["blocks"] <= 92


def test_autotune_result_before_any_run(qs):
    c = qs.Circuit(cg.random_circuit(4, 5, 4, seed=3, cu3_prob=0.1))
    assert c.autotune_result(20, qs.C64) == (0, 6, 0, 0, 0.0)
    assert c.autotune_result(12, qs.C64)[:2] == (0, 4)  # tile sizes 11, 12
    assert c.autotune_result(20, qs.C128)[:2] == (0, 3)  # block widths 2..4
    with pytest.raises(qs.QSError) as e:
        c.autotune_result(20, 9)
    assert e.value.status == -1
    # without measurements the plan is the greedy one
    assert (c.plan_info(20, qs.C64, qs.PLAN_AUTOTUNE) == c.plan_info(20, qs.C64, qs.PLAN_GREEDY))


@pytest.mark.parametrize("struct,cname", [("RunOpts", "qs_run_opts"), ("TrajStats", "qs_traj_stats"),
                                          ("SingleInfo", "qs_single_info"), ("ScriptInfo", "qs_script_info")])
def test_binding_structs_match_header(qs, tmp_path, struct, cname):
    """Each ctypes structure of the binding mirrors its C struct field by
    field (offsets and size from a C program built against include/qs.h),
    and the candidate count of tile orders agrees."""
    import ctypes
    import subprocess
    cls = getattr(qs, struct)
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"qs.h\"\nint main(void) {\n"
                   + "".join('printf("%%zu\\n", offsetof(%s, %s));\n' % (cname, f) for f in fields)
                   + 'printf("%%zu\\n%%d\\n", sizeof(%s), QS_TILE_ORDERS);\nreturn 0;\n}\n' % cname)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(cls, f).offset for f in fields] + [ctypes.sizeof(cls), qs.TILE_ORDERS]
    assert got == want


def _crossing_gates(ops, part_a):
    return sum(1 for o in ops if o.kind == "gate"
               and {(part_a >> q) & 1 for q in tuple(o.targets) + tuple(o.controls)} == {0, 1})


def test_partial_cut_counts_on_grid_circuits(qs):
    """Partial-amplitude mode (Eq. 4): every CZ across the dividing line is one
    cut.  An 8 x 5 grid (40 qubits) at depth 8 divided between rows 3 and 4 is
    crossed by the vertical pairs at odd rows, in layers 3 and 7: 2 x 5 CZ.  A
    6 x 5 grid at depth 8 divided between rows 2 and 3 is crossed in layers 1
    and 5 (vertical pairs at even rows)."""
    for rows, cols, depth, top_rows, want in [(8, 5, 8, 4, 10), (6, 5, 8, 3, 10), (6, 5, 12, 3, 15)]:
        ops = cg.random_circuit(rows, cols, depth, seed=6001)
        n, part_a = rows * cols, (1 << (top_rows * cols)) - 1
        assert _crossing_gates(ops, part_a) == want
        assert qs.Circuit(ops).partial_cuts(n, part_a) == want


def test_partial_cut_forms_and_rejections(qs):
    """Crossing gates that are cut (controlled gates with their targets on one
    side, diagonal gates with one qubit on one side, CONTROL groups) and the
    ones that are rejected (SWAP, a diagonal with two qubits on each side,
    noise, more than QS_PARTIAL_MAX_CUTS cuts)."""
    n, A = 6, 0b000111
    rng = np.random.default_rng(3)
    X = cg.PX
    d3 = np.diag(np.exp(1j * rng.uniform(0, 6.28, 8)))
    d4 = np.diag(np.exp(1j * rng.uniform(0, 6.28, 16)))
    swap = np.eye(4)[[0, 2, 1, 3]]
    ok = [([cg.Gate((4,), (1,), X)], 1), ([cg.Gate((1,), (4,), X)], 1),
          ([cg.Gate((0, 5), (), cg.CZ_GATE)], 1), ([cg.Gate((3,), (0, 1), X)], 1),
          ([cg.Gate((3,), (0, 4), X)], 1), ([cg.Gate((2, 3, 4), (), d3)], 1),
          ([cg.Gate((0, 3), (), np.eye(4))], 0),
          ([cg.Marker("control", 0), cg.Gate((3,), (), cg.H_GATE), cg.Gate((4,), (), cg.T_GATE),
            cg.Marker("endcontrol")], 2)]
    for ops, want in ok:
        assert qs.Circuit(ops).partial_cuts(n, A) == want
    bad = [[cg.Gate((0, 3), (), swap)], [cg.Gate((0, 1, 3, 4), (), d4)],
           [cg.Gate((0,), (), cg.H_GATE), cg.Noise((0,), cg.kraus_depolarizing(0.1))],
           [cg.Gate((0, 5), (), cg.CZ_GATE)] * 25]
    for ops in bad:
        with pytest.raises(qs.QSError) as e:
            qs.Circuit(ops).partial_cuts(n, A)
        assert e.value.status == -6
    c = qs.Circuit([cg.Gate((7,), (), cg.H_GATE)])
    with pytest.raises(qs.QSError) as e:
        c.partial_cuts(n, A)
    assert e.value.status == -2
    c = qs.Circuit([cg.Gate((0,), (), cg.H_GATE)])
    for nn, part in [(n, 0), (n, 0b111111), (n, 1 << 6), (1, 1), (63, 1)]:
        with pytest.raises(qs.QSError) as e:
            c.partial_cuts(nn, part)
        assert e.value.status == -1
    with pytest.raises(qs.QSError) as e:
        c.partial_cuts(40, (1 << 38) - 1)  # part A of 38 qubits
    assert e.value.status == -6


# --------------------------------------------------------------- scripts --

SCRIPT_ALL = """# every App. A-1 instruction
QINIT 4
CREG 2
H 0
X 1
Y 2
Z 3
S 0
T 1
RX 2, "pi/3"
RY 3, "-pi/4"
RZ 0, "3*pi/4"
U4 1, "0.1, (1+1)*pi/8, -0.7, 1e-1"
CNOT 0, 2
CZ 1, 3
CR 2, 0, "pi/2"
SWAP 1, 2
ISWAP 0, 3
TOFFOLI 0, 1, 3
DAGGER
H 2
CR 2, 3, "pi/5"
DAGGER
T 0
ENDDAGGER
ENDDAGGER
CONTROL 3
RY 0, "0.3"
CONTROL 2
X 1
ENDCONTROL 2
ENDCONTROL 3
H 0
H 1
H 2
H 3
"""


def _golden_script():
    with open(os.path.join(ROOT, "tests", "golden", "appA2_example.txt")) as f:
        text = f.read()
    return text, text.split("%Output")[0]


def test_script_parse_counts_and_info(qs):
    """The App. A-1 parser builds the circuit the test-side reader builds for
    the App. A-2 example (same gate counts after DAGGER expansion) and
    reports QINIT, CREG and the PMEASURE qubits."""
    from tests import appa_script
    full, text = _golden_script()
    n, ops, pm, _ = appa_script.parse(full, oracle.named_gate)
    c, info = qs.script_parse(text)
    assert info == {"n": n, "creg": 3, "measures": 0, "pmeasure": pm}
    assert c.counts() == qs.Circuit(ops).counts()
    c, info = qs.script_parse(SCRIPT_ALL)
    n, ops, _, _ = appa_script.parse(SCRIPT_ALL, oracle.named_gate)
    assert info["n"] == n == 4 and info["pmeasure"] == []
    assert c.counts() == qs.Circuit(ops).counts() == (25, 0, 25)


def test_script_errors_name_the_line(qs):
    cases = [("QINIT 2\nH 0\nFOO 1\n", -1, "line 3"), ("QINIT 2\nH 2\n", -2, "line 2"),
             ("H 0\n", -1, "line 1"), ("QINIT 2\nRX 0, \"pi/\"\n", -1, "line 2"),
             ("QINIT 2\nCREG 1\nDAGGER\nMEASURE 0, $0\nENDDAGGER\n", -6, "line 4"),
             ("QINIT 2\nPMEASURE 0\nH 1\n", -1, "line 3"), ("QINIT 2\nCREG 1\nMEASURE 0, $1\n", -2, "line 3"),
             ("QINIT 3\nCONTROL 0\nH 1\nENDCONTROL 2\n", -1, "line 4"), ("QINIT 2\nDAGGER\nH 0\n", -1, "line 2"),
             ("QINIT 2\nCNOT 0\n", -1, "line 2"), ("QINIT 2\nMEASURE 0, 0\n", -1, "line 2"),
             ("QINIT 2\nPMEASURE 1, 1\n", -2, "line 2"), ("QINIT 40\n", -1, "line 1")]
    for text, status, where in cases:
        with pytest.raises(qs.QSError) as e:
            qs.script_parse(text)
        assert e.value.status == status, text
        assert qs.last_error().startswith(where + ":"), (text, qs.last_error())


# ------------------------------------------------ single-amplitude mode --


def test_single_graph_vertex_rules(qs):
    """Fig. 2: a diagonal gate keeps its qubits' vertices (a), (c); any other
    gate adds one vertex per target (b), (d), and a control keeps its vertex.
    Every qubit's first vertex is fixed to 0 and its last to the measured bit
    (a qubit whose first vertex is also its last is fixed once)."""
    n = 5
    h = cg.H_GATE
    cnot = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
    diag_only = [cg.Gate((q,), (), cg.T_GATE) for q in range(n)] + \
        [cg.Gate((0, 1), (), cg.CZ_GATE), cg.Gate((2, 4), (), cg.CZ_GATE)]
    i = qs.Circuit(diag_only).single_plan(n)
    assert i["vertices"] == n and i["fixed"] == n and i["tensors"] == len(diag_only)
    dense = [cg.Gate((q,), (), h) for q in range(n)]
    i = qs.Circuit(dense).single_plan(n)
    assert i["vertices"] == 2 * n and i["fixed"] == 2 * n and i["tensors"] == n
    # CNOT: the control keeps its vertex, the target gets one; a dense
    # two-qubit gate gets two; CU3 (controlled U3) one
    two = [cg.Gate((0, 1), (), cnot), cg.Gate((2, 3), (), cg.random_unitary(4, np.random.default_rng(1))),
           cg.Gate((4,), (1,), cg.u3(0.3, 0.2, 0.1))]
    i = qs.Circuit(two).single_plan(n)
    assert i["vertices"] == n + 1 + 2 + 1
    # identity gates are no edges
    i = qs.Circuit([cg.Gate((q,), (), np.eye(2)) for q in range(n)]).single_plan(n)
    assert i["vertices"] == n and i["tensors"] == 0 and i["merges"] == 0


def test_single_graph_counts_on_workload_circuits(qs):
    """On the grid random circuits (T and CZ diagonal, the other one-qubit
    gates and CU3 dense on one target) the vertex count is n plus the
    non-diagonal one-qubit gates; slicing fixes that many more vertices and
    multiplies the graphs, and planning is deterministic."""
    for rows, cols, depth, cu3 in ((4, 4, 8, 0.1), (7, 7, 10, 0.0), (6, 10, 10, 0.0)):
        n = rows * cols
        ops = cg.random_circuit(rows, cols, depth, seed=77, cu3_prob=cu3)
        dense = sum(1 for o in ops if o.kind == "gate" and o.name not in ("t", "cz"))
        c = qs.Circuit(ops)
        i0 = c.single_plan(n)
        assert i0["vertices"] == n + dense
        assert i0["fixed"] == 2 * n and i0["sliced"] == 0 and i0["batch"] == 1
        assert i0["tensors"] >= sum(1 for o in ops if o.kind == "gate")
        i4 = c.single_plan(n, 4)
        assert i4["sliced"] == 4 and i4["fixed"] == 2 * n + 4 and i4["batch"] == 16
        assert c.single_plan(n) == i0


def test_single_validation(qs):
    c = qs.Circuit([cg.Gate((0,), (), cg.H_GATE)])
    for n, ns, st in ((0, 0, -1), (63, 0, -1), (2, -1, -1), (2, 17, -1)):
        with pytest.raises(qs.QSError) as e:
            c.single_plan(n, ns)
        assert e.value.status == st
    with pytest.raises(qs.QSError) as e:
        qs.Circuit([cg.Gate((5,), (), cg.H_GATE)]).single_plan(3)
    assert e.value.status == -2
    noisy = qs.Circuit([cg.Gate((0,), (), cg.I2), cg.Noise((0,), cg.kraus_depolarizing(0.1))])
    with pytest.raises(qs.QSError) as e:
        noisy.single_plan(2)
    assert e.value.status == -6
    with pytest.raises(qs.QSError) as e:
        c.single_amplitudes(2, [4])  # bit 2 set on a 2-qubit circuit: rejected before any device work
    assert e.value.status == -2


def test_profile_source_hash_ignores_comments_only(tmp_path):
    """Stored counter readings are keyed by a hash of the profiled device
    sources with comments and layout left out: a comment edit keeps the
    key, a change to the code changes it."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    csrc = tmp_path / "paper_2008_07140_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.h").write_text("// header\nconstexpr int kW = 4;  /* width */\n")
    (csrc / "k.hip").write_text('#include "k.h"\n__global__ void k(int *p) { p[0] = kW; }  // store\n')
    h0 = bench.source_hash(("k.hip",), root=str(tmp_path))
    (csrc / "k.h").write_text("/* a longer\n   header comment */\nconstexpr int kW = 4;\n")
    (csrc / "k.hip").write_text('#include "k.h"\n// the kernel\n__global__ void k(int *p)\n{\n    p[0] = kW;\n}\n')
    assert bench.source_hash(("k.hip",), root=str(tmp_path)) == h0
    (csrc / "k.h").write_text("constexpr int kW = 5;\n")
    assert bench.source_hash(("k.hip",), root=str(tmp_path)) != h0
