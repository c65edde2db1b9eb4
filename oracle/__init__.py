"""ctypes wrapper for the FP64 CPU oracle (qs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  It reads
circuits produced by the seeded generator by duck typing (attributes
``kind``, ``targets``, ``controls``, ``matrix``, ``kraus``, ``qubit``) and
shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP over the outer loops)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            P = C.c_void_p
            i, d, u64 = C.c_int, C.c_double, C.c_uint64
            L.or_num_threads.argtypes = []
            L.or_num_threads.restype = i
            L.or_set_threads.argtypes = [i]
            L.or_init.argtypes = [P, i]
            L.or_norm2.argtypes = [P, i]
            L.or_norm2.restype = d
            L.or_apply.argtypes = [P, i, P, i, P, i, P]
            L.or_probabilities.argtypes = [P, i, P, i, P]
            L.or_named_gate.argtypes = [C.c_char_p, P, P]
            L.or_philox4x32_10.argtypes = [P, P, P]
            L.or_uniform.argtypes = [u64, u64, u64]
            L.or_uniform.restype = d
            L.or_apply_noisy.argtypes = [P, i, P, i, P, P, i, d, P, P, P]
            L.or_dm_apply.argtypes = [P, i, P, i, P, i, P]
            L.or_dm_channel.argtypes = [P, i, P, i, P, i]
            L.or_dm_expect_z.argtypes = [P, i, P]
            L.or_expect_z.argtypes = [P, i, P]
            L.or_run.argtypes = [P, i, i, P, P, P, P, P, P, P, P, u64, u64, P]
            L.or_mlp_num_params.argtypes = [i, i]
            L.or_mlp_num_params.restype = C.c_size_t
            L.or_mlp_forward_backward.argtypes = [P, i, i, i, P, P, P, P]
            L.or_mlp_forward_backward.restype = d
            _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _ints(xs):
    return np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))


def _cmat(m):
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128))


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(k: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only)."""
    lib().or_set_threads(int(k))


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_init(_ptr(psi), n)
    return psi


def norm2(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return lib().or_norm2(_ptr(psi), n)


def apply(psi: np.ndarray, targets, controls, m) -> None:
    n = int(psi.size).bit_length() - 1
    t, c, mm = _ints(targets), _ints(controls), _cmat(m)
    rc = lib().or_apply(_ptr(psi), n, _ptr(t), len(t), _ptr(c), len(c), _ptr(mm))
    if rc:
        raise ValueError("oracle: invalid qubits")


def probabilities(psi: np.ndarray, qubits) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    q = _ints(qubits)
    out = np.empty(1 << len(q), dtype=np.float64)
    if lib().or_probabilities(_ptr(psi), n, _ptr(q), len(q), _ptr(out)):
        raise ValueError("oracle: invalid qubits")
    return out


def named_gate(name: str, params=()) -> np.ndarray:
    m = np.zeros(64, dtype=np.complex128)
    p = np.ascontiguousarray(np.asarray(list(params) + [0.0] * 8, dtype=np.float64))
    k = lib().or_named_gate(name.encode(), _ptr(p), _ptr(m))
    if k < 0:
        raise KeyError(name)
    d = 1 << k
    return m[: d * d].reshape(d, d).copy()


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return [int(v) for v in o]


def uniform(seed: int, traj: int, site: int) -> float:
    return lib().or_uniform(seed, traj, site)


def apply_noisy(psi, targets, m, kraus, u):
    """Sec. 2.4 noisy gate; returns (chosen branch, p_chosen, all p_b)."""
    n = int(psi.size).bit_length() - 1
    t, mm, kk = _ints(targets), _cmat(m), _cmat(kraus)
    nk = kk.shape[0]
    ch = np.zeros(1, dtype=np.int32)
    pc = np.zeros(1, dtype=np.float64)
    probs = np.zeros(nk, dtype=np.float64)
    rc = lib().or_apply_noisy(_ptr(psi), n, _ptr(t), len(t), _ptr(mm), _ptr(kk), nk, u,
                              _ptr(ch), _ptr(pc), _ptr(probs))
    if rc:
        raise ValueError("oracle: noisy gate failed (%d)" % rc)
    return int(ch[0]), float(pc[0]), probs


def dm_zero(n: int) -> np.ndarray:
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def dm_apply(rho, targets, controls, m) -> None:
    n = int(rho.shape[0]).bit_length() - 1
    t, c, mm = _ints(targets), _ints(controls), _cmat(m)
    if lib().or_dm_apply(_ptr(rho), n, _ptr(t), len(t), _ptr(c), len(c), _ptr(mm)):
        raise ValueError("oracle: invalid qubits")


def dm_channel(rho, targets, kraus) -> None:
    n = int(rho.shape[0]).bit_length() - 1
    t, kk = _ints(targets), _cmat(kraus)
    if lib().or_dm_channel(_ptr(rho), n, _ptr(t), len(t), _ptr(kk), kk.shape[0]):
        raise ValueError("oracle: invalid qubits")


def dm_expect_z(rho) -> np.ndarray:
    n = int(rho.shape[0]).bit_length() - 1
    out = np.zeros(n, dtype=np.float64)
    lib().or_dm_expect_z(_ptr(rho), n, _ptr(out))
    return out


def expect_z(psi) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    out = np.zeros(n, dtype=np.float64)
    lib().or_expect_z(_ptr(psi), n, _ptr(out))
    return out


def dm_run(n: int, ops) -> np.ndarray:
    """Density-matrix evolution of a gate/noise list without groups (n <= 10)."""
    rho = dm_zero(n)
    for o in ops:
        if o.kind == "gate":
            dm_apply(rho, o.targets, o.controls, o.matrix)
        elif o.kind == "noise":
            dm_channel(rho, o.targets, o.kraus)
        else:
            raise ValueError("dm_run: groups are not supported")
    return rho


_KIND = {"gate": 0, "noise": 1, "dagger": 2, "enddagger": 3, "control": 4, "endcontrol": 5}


def _marshal(ops):
    kind, nt, nc, q_off, nk, mat_off = [], [], [], [], [], []
    qubits, mats = [], []
    moff = 0
    for o in ops:
        k = _KIND[o.kind]
        kind.append(k)
        q_off.append(len(qubits))
        mat_off.append(moff)
        if k == 0:
            m = _cmat(o.matrix)
            nt.append(len(o.targets)); nc.append(len(o.controls)); nk.append(0)
            qubits += list(o.targets) + list(o.controls)
            mats.append(m.reshape(-1)); moff += m.size
        elif k == 1:
            kr = _cmat(o.kraus)
            nt.append(len(o.targets)); nc.append(0); nk.append(kr.shape[0])
            qubits += list(o.targets)
            mats.append(kr.reshape(-1)); moff += kr.size
        elif k == 4:
            nt.append(0); nc.append(0); nk.append(0)
            qubits.append(int(o.qubit))
        else:
            nt.append(0); nc.append(0); nk.append(0)
    flat = np.concatenate(mats) if mats else np.zeros(1, dtype=np.complex128)
    mats_d = np.ascontiguousarray(np.stack([flat.real, flat.imag], axis=1).reshape(-1))
    arr = lambda x: np.ascontiguousarray(np.asarray(x if x else [0], dtype=np.int32))
    return (len(kind), arr(kind), arr(nt), arr(nc), arr(q_off), arr(qubits), arr(mat_off),
            mats_d, arr(nk))


def run(n: int, ops, seed: int = 0, traj: int = 0, psi=None):
    """Run a circuit from |0...0> (or from psi, modified in place).

    Returns (psi, chosen) where chosen lists the Kraus branch of every noise
    site in order."""
    if psi is None:
        psi = zero_state(n)
    nops, kind, nt, nc, q_off, qubits, mat_off, mats, nk = _marshal(ops)
    nsites = sum(1 for o in ops if o.kind == "noise")
    chosen = np.zeros(max(nsites, 1), dtype=np.int32)
    rc = lib().or_run(_ptr(psi), n, nops, _ptr(kind), _ptr(nt), _ptr(nc), _ptr(q_off),
                      _ptr(qubits), _ptr(mat_off), _ptr(mats), _ptr(nk), seed, traj,
                      _ptr(chosen))
    if rc:
        raise ValueError("oracle: run failed (%d)" % rc)
    return psi, chosen[:nsites]


def mlp_num_params(f: int, h: int) -> int:
    return int(lib().or_mlp_num_params(f, h))


def mlp_forward_backward(params, f, h, x, t=None):
    """Returns (y, loss, grad) in FP64; grad is None when t is None."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = x.shape[0]
    y = np.zeros(b, dtype=np.float64)
    grad = np.zeros(mlp_num_params(f, h), dtype=np.float64) if t is not None else None
    tt = np.ascontiguousarray(t, dtype=np.float64) if t is not None else None
    loss = lib().or_mlp_forward_backward(_ptr(params), f, h, b, _ptr(x), _ptr(tt), _ptr(y),
                                         _ptr(grad))
    return y, loss, grad
