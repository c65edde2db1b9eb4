"""Seeded synthetic circuit generator.

Input data only: this module draws random circuits and writes out the gate
and Kraus matrices that describe them.  It contains none of the simulation
arithmetic (no state, no gate application, no sampling of noise branches);
the HIP library and the FP64 oracle each consume its output independently.

Workload shape follows the random-circuit benchmarks of Sec. 3.1 (random
quantum circuits on a qubit grid, layers of single-qubit gates followed by
nearest-neighbour CZ gates); Google's circuit files are not used.  Qubit
q = r * C + c on an R x C grid.  Layer l applies one single-qubit gate to every
qubit, drawn uniformly from {sqrt(X), sqrt(Y), sqrt(W), T, U3}, then CZ on
the pair pattern l mod 4 (horizontal pairs at even columns, vertical pairs at
even rows, horizontal at odd columns, vertical at odd rows).

Gate matrices: App. A-1 prints H, X, Y, Z, S, T, RX/RY/RZ, U4, CNOT, CZ, CR,
SWAP, iSWAP, TOFFOLI.  sqrt(P) for P in {X, Y, W = (X+Y)/sqrt(2)} is the
principal root ((1+i) I + (1-i) P) / 2 (exact because P^2 = I).  U3 is the
OpenQASM 2 form.  Kraus sets are Eq. 5 of Sec. 2.4; two-qubit sets are the
Kronecker products of Sec. 2.4.

Multi-qubit matrices are row-major with targets[0] as the most significant
bit of the row index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

C128 = np.complex128


@dataclass(frozen=True)
class Gate:
    targets: Tuple[int, ...]
    controls: Tuple[int, ...]
    matrix: np.ndarray  # (2^nt, 2^nt) complex128
    name: str = ""
    kind: str = field(default="gate", init=False)


@dataclass(frozen=True)
class Noise:
    """Kraus channel acting right after the preceding gate (same targets)."""

    targets: Tuple[int, ...]
    kraus: np.ndarray  # (nk, 2^nt, 2^nt) complex128
    name: str = ""
    kind: str = field(default="noise", init=False)


@dataclass(frozen=True)
class Marker:
    """DAGGER / ENDDAGGER / CONTROL q / ENDCONTROL group markers (App. A-1)."""

    kind: str  # "dagger" | "enddagger" | "control" | "endcontrol"
    qubit: int = -1


# ---------------------------------------------------------------- matrices --

I2 = np.eye(2, dtype=C128)
PX = np.array([[0, 1], [1, 0]], dtype=C128)
PY = np.array([[0, -1j], [1j, 0]], dtype=C128)
PZ = np.array([[1, 0], [0, -1]], dtype=C128)
PW = (PX + PY) / math.sqrt(2.0)


def sqrt_pauli(p: np.ndarray) -> np.ndarray:
    return ((1 + 1j) * I2 + (1 - 1j) * p) / 2


SQRT_X = sqrt_pauli(PX)
SQRT_Y = sqrt_pauli(PY)
SQRT_W = sqrt_pauli(PW)
T_GATE = np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=C128)
H_GATE = np.array([[1, 1], [1, -1]], dtype=C128) / math.sqrt(2.0)
CZ_GATE = np.diag([1, 1, 1, -1]).astype(C128)


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array(
        [[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
        dtype=C128,
    )


def rz(theta: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(C128)


def ry(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=C128)


def rx(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=C128)


# ------------------------------------------------------------- Kraus sets --
# Eq. 5.  For the three flip channels p is the weight of the identity branch
# (noise vanishes as p -> 1); for the damping and depolarizing channels the
# noise vanishes as p -> 0.


def kraus_bit_flip(p: float) -> np.ndarray:
    return np.stack([math.sqrt(p) * I2, math.sqrt(1 - p) * PX])


def kraus_phase_flip(p: float) -> np.ndarray:
    return np.stack([math.sqrt(p) * I2, math.sqrt(1 - p) * PZ])


def kraus_bit_phase_flip(p: float) -> np.ndarray:
    return np.stack([math.sqrt(p) * I2, math.sqrt(1 - p) * PY])


def kraus_amplitude_damping(p: float) -> np.ndarray:
    k1 = np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=C128)
    k2 = np.array([[0, math.sqrt(p)], [0, 0]], dtype=C128)
    return np.stack([k1, k2])


def kraus_phase_damping(p: float) -> np.ndarray:
    k1 = np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=C128)
    k2 = np.array([[0, 0], [0, math.sqrt(p)]], dtype=C128)
    return np.stack([k1, k2])


def kraus_depolarizing(p: float) -> np.ndarray:
    return np.stack(
        [math.sqrt(1 - 3 * p / 4) * I2, math.sqrt(p) / 2 * PX, math.sqrt(p) / 2 * PY,
         math.sqrt(p) / 2 * PZ]
    )


def kraus_kron(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Two-qubit set {K_i (x) M_j} in the order K_1M_1, K_1M_2, ..., K_2M_1, ..."""
    return np.stack([np.kron(ka, mb) for ka in a for mb in b])


KRAUS_SETS = {
    "bit_flip": kraus_bit_flip,
    "phase_flip": kraus_phase_flip,
    "bit_phase_flip": kraus_bit_phase_flip,
    "amplitude_damping": kraus_amplitude_damping,
    "phase_damping": kraus_phase_damping,
    "depolarizing": kraus_depolarizing,
}


# ------------------------------------------------------------ grid layout --


def grid_shape(n: int) -> Tuple[int, int]:
    """R = the largest divisor of n not above sqrt(n), C = n / R."""
    r = max(d for d in range(1, int(math.isqrt(n)) + 1) if n % d == 0)
    return r, n // r


def cz_pairs(rows: int, cols: int, pattern: int) -> List[Tuple[int, int]]:
    pairs = []
    if pattern in (0, 2):
        c0 = 0 if pattern == 0 else 1
        for r in range(rows):
            for c in range(c0, cols - 1, 2):
                pairs.append((r * cols + c, r * cols + c + 1))
    else:
        r0 = 0 if pattern == 1 else 1
        for r in range(r0, rows - 1, 2):
            for c in range(cols):
                pairs.append((r * cols + c, (r + 1) * cols + c))
    return pairs


ONE_QUBIT_KINDS = ("sqrt_x", "sqrt_y", "sqrt_w", "t", "u3")


def _one_qubit(rng: np.random.Generator) -> Tuple[str, np.ndarray]:
    k = ONE_QUBIT_KINDS[int(rng.integers(0, len(ONE_QUBIT_KINDS)))]
    if k == "sqrt_x":
        return k, SQRT_X
    if k == "sqrt_y":
        return k, SQRT_Y
    if k == "sqrt_w":
        return k, SQRT_W
    if k == "t":
        return k, T_GATE
    th, ph, la = rng.uniform(0.0, 2 * math.pi, size=3)
    return k, u3(th, ph, la)


def random_circuit(rows: int, cols: int, depth: int, seed: int, cu3_prob: float = 0.0,
                   dep1: float = 0.0, dep2: float = 0.0, damping: float = 0.0) -> list:
    """Layered grid random circuit.

    cu3_prob: probability that a single-qubit slot becomes a controlled-U3
    with the control drawn uniformly among the other qubits.
    dep1 / dep2: depolarizing p after every single-qubit gate / after every CZ
    (two-qubit set = Kronecker product of two one-qubit sets).
    damping: amplitude-damping p applied to every qubit, in ascending order,
    after the CZ sublayer of each layer (as a noisy identity gate).
    """
    n = rows * cols
    rng = np.random.default_rng(seed)
    ops: list = []
    k1 = kraus_depolarizing(dep1) if dep1 > 0 else None
    k2 = kraus_kron(kraus_depolarizing(dep2), kraus_depolarizing(dep2)) if dep2 > 0 else None
    kd = kraus_amplitude_damping(damping) if damping > 0 else None
    for layer in range(depth):
        for q in range(n):
            name, m = _one_qubit(rng)
            if cu3_prob > 0 and rng.random() < cu3_prob:
                th, ph, la = rng.uniform(0.0, 2 * math.pi, size=3)
                c = int(rng.integers(0, n - 1))
                c = c if c < q else c + 1
                ops.append(Gate((q,), (c,), u3(th, ph, la), "cu3"))
                continue
            ops.append(Gate((q,), (), m, name))
            if k1 is not None:
                ops.append(Noise((q,), k1, "depolarizing"))
        for a, b in cz_pairs(rows, cols, layer % 4):
            ops.append(Gate((a, b), (), CZ_GATE, "cz"))
            if k2 is not None:
                ops.append(Noise((a, b), k2, "depolarizing2"))
        if kd is not None:
            for q in range(n):
                ops.append(Gate((q,), (), I2, "id"))
                ops.append(Noise((q,), kd, "amplitude_damping"))
    return ops


def count_gates(ops: Sequence) -> int:
    """Logical gates (identity carriers of idle noise are not counted)."""
    return sum(1 for o in ops if o.kind == "gate" and o.name != "id")


# ------------------------------------------------------------ workloads --

WORKLOADS = {
    # name: (rows, cols, depth, seed, cu3_prob)
    "rqc16_d20": (4, 4, 20, 1001, 0.0),
    "rqc30_d40": (6, 5, 40, 2001, 0.10),
    "rqc32_d32": (8, 4, 32, 3001, 0.0),
    "rqc34_d24": (17, 2, 24, 5001, 0.0),
}


def workload(name: str) -> Tuple[int, list]:
    rows, cols, depth, seed, cu3 = WORKLOADS[name]
    return rows * cols, random_circuit(rows, cols, depth, seed, cu3_prob=cu3)


def trajectory_batch(count: int, seed: int = 4001, nmin: int = 14, nmax: int = 22,
                     depth: int = 24, dep1: float = 1e-3, dep2: float = 1e-2,
                     damping: float = 5e-4) -> List[Tuple[int, list]]:
    """`count` noisy random circuits of uneven width n ~ U{nmin..nmax}."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        r, c = grid_shape(n)
        out.append((n, random_circuit(r, c, depth, seed + t, dep1=dep1, dep2=dep2,
                                      damping=damping)))
    return out


def random_state(n: int, seed: int) -> np.ndarray:
    """A normalised random complex128 state (Gaussian entries)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(C128)


def random_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-ish random unitary from the QR factor of a complex Gaussian matrix."""
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph).astype(C128)
