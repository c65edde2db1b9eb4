"""ctypes binding of libqs.so (include/qs.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; this module
converts numpy arrays and circuit objects to the C ABI and raises
``QSError`` on a negative status.  The library must have been built
(``python -m paper_2008_07140_amd.build``); importing this module without
it raises immediately instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libqs.so is not built: run `python -m paper_2008_07140_amd.build`")

_lib = C.CDLL(LIB_PATH)

C64, C128 = 1, 2
COST_FEATURES = 16
MLP_HIDDEN = 64
PLAN_UNFUSED, PLAN_GREEDY, PLAN_LEARNED, PLAN_AUTOTUNE = 0, 1, 2, 3
TILE_ORDERS = 4  # candidate tile orders of a sweep (RunOpts.tile_order 1..TILE_ORDERS; 0 = measured)
(K_INIT, K_DENSE1, K_DENSE2, K_DENSE3, K_DENSEN, K_PHASE, K_FUSED, K_TILE, K_REDUCE,
 K_OTHER) = range(10)
KERNEL_NAMES = ["init", "dense1", "dense2", "dense3", "denseN", "phase", "fused", "tile",
                "reduce", "other"]

STATUS = {0: "QS_OK", -1: "QS_E_INVAL", -2: "QS_E_RANGE", -3: "QS_E_NOMEM", -4: "QS_E_DEVICE",
          -5: "QS_E_ZERO_NORM", -6: "QS_E_UNSUPPORTED"}


class QSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class RunOpts(C.Structure):
    _fields_ = [("plan", C.c_int), ("k_max", C.c_int), ("seed", C.c_uint64),
                ("traj", C.c_uint64), ("chosen", C.POINTER(C.c_int64)),
                ("chosen_len", C.c_int64), ("tile_qubits", C.c_int), ("tile_order", C.c_int),
                ("direct_launch", C.c_int)]


class TrajStats(C.Structure):
    _fields_ = [("passes", C.c_int), ("graphs", C.c_int), ("chunk", C.c_int), ("host_sampled", C.c_int),
                ("jumps", C.c_int64),
                ("launches", C.c_int64), ("graph", C.c_int), ("tile_qubits", C.c_int),
                ("k_max", C.c_int), ("max_outer", C.c_int), ("autotune_tried", C.c_int),
                ("autotune_candidates", C.c_int), ("seconds", C.c_double),
                ("host_seconds", C.c_double), ("device_seconds", C.c_double)]


class SingleInfo(C.Structure):
    _fields_ = [("vertices", C.c_int), ("tensors", C.c_int), ("fixed", C.c_int), ("sliced", C.c_int),
                ("merges", C.c_int), ("max_rank", C.c_int), ("flops", C.c_double),
                ("peak_bytes", C.c_double), ("batch", C.c_int), ("own_low", C.c_int)]


class ScriptInfo(C.Structure):
    _fields_ = [("n", C.c_int), ("creg", C.c_int), ("measures", C.c_int), ("pmeasure_n", C.c_int),
                ("pmeasure", C.c_int * 36)]


P, I, D, U64, I64, SZ = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_int64, C.c_size_t
PP = C.POINTER(C.c_void_p)
_sig = {
    "qs_create": ([I, I, PP], I),
    "qs_create_from_buffer": ([I, I, P, SZ, P, PP], I),
    "qs_destroy": ([P], I),
    "qs_reset": ([P], I),
    "qs_set_amplitudes": ([P, P], I),
    "qs_info": ([P, P, P, PP, PP], I),
    "qs_synchronize": ([P], I),
    "qs_set_memory_limit": ([SZ], I),
    "qs_apply_gate": ([P, P, I, P, I, P], I),
    "qs_apply_noisy_gate": ([P, P, I, P, I, P, P, I, D, P, P], I),
    "qs_circuit_create": ([PP], I),
    "qs_circuit_destroy": ([P], I),
    "qs_circuit_append_gate": ([P, P, I, P, I, P], I),
    "qs_circuit_append_noise": ([P, P, I, P, I], I),
    "qs_circuit_begin_dagger": ([P], I),
    "qs_circuit_end_dagger": ([P], I),
    "qs_circuit_begin_control": ([P, I], I),
    "qs_circuit_end_control": ([P], I),
    "qs_circuit_counts": ([P, P, P, P], I),
    "qs_run_circuit": ([P, P, C.POINTER(RunOpts)], I),
    "qs_circuit_plan_info": ([P, I, I, C.POINTER(RunOpts), P, P, P], I),
    "qs_amplitudes": ([P, P, SZ, P], I),
    "qs_probabilities": ([P, P, I, P], I),
    "qs_probabilities_noalloc": ([P, I, I, P, I, P, P], I),
    "qs_norm": ([P, P], I),
    "qs_expect_z": ([P, P], I),
    "qs_run_trajectories": ([P, P, I, I, U64, C.POINTER(RunOpts), P, P], I),
    "qs_trajectory_stats": ([C.POINTER(TrajStats)], I),
    "qs_remap_pack": ([P, I, P, P], I),
    "qs_remap_unpack": ([P, I, P, P], I),
    "qs_partial_amplitudes": ([P, I, I, U64, P, SZ, P, C.POINTER(RunOpts), P], I),
    "qs_partial_cuts": ([P, I, U64, P], I),
    "qs_single_amplitudes": ([P, I, P, SZ, I, P, C.POINTER(SingleInfo)], I),
    "qs_single_plan": ([P, I, I, C.POINTER(SingleInfo)], I),
    "qs_script_parse": ([C.c_char_p, PP, C.POINTER(ScriptInfo)], I),
    "qs_script_run": ([C.c_char_p, I, U64, I, P, I, P, SZ, C.POINTER(ScriptInfo)], I),
    "qs_philox_uniform": ([U64, U64, U64], D),
    "qs_philox4x32_10": ([P, P, P], None),
    "qs_profile_enable": ([P, I], I),
    "qs_profile_reset": ([P], I),
    "qs_profile_query": ([P, I, P, P, P, P], I),
    "qs_mlp_forward": ([P, I, I, P, I64, P], I),
    "qs_mlp_grad": ([P, I, I, P, P, I64, P, P], I),
    "qs_mlp_train": ([P, I, I, P, P, I64, I, I, C.c_float, U64, P], I),
    "qs_profile_samples": ([P, P, P, I64, P], I),
    "qs_cost_model_set": ([P, I, I], I),
    "qs_circuit_autotune_result": ([P, I, I, P, P, P, P, P], I),
    "qs_last_error": ([], C.c_char_p),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = sorted(_sig)


def lib():
    return _lib


def last_error() -> str:
    return _lib.qs_last_error().decode()


def _check(st: int):
    if st != 0:
        raise QSError(st, last_error())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _ints(xs) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))


def _mat(m) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    return a.view(np.float64).reshape(-1)


def set_memory_limit(nbytes: int) -> None:
    _check(_lib.qs_set_memory_limit(nbytes))


def philox_uniform(seed: int, traj: int, site: int) -> float:
    return _lib.qs_philox_uniform(seed, traj, site)


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _lib.qs_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return [int(v) for v in o]


def mlp_num_params(f: int, h: int = MLP_HIDDEN) -> int:
    return h * f + h + h * h + h + h + 1


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def mlp_forward(params, x, f: int = COST_FEATURES, h: int = MLP_HIDDEN) -> np.ndarray:
    p, xx = _f32(params), _f32(x).reshape(-1, f)
    y = np.empty(xx.shape[0], dtype=np.float32)
    _check(_lib.qs_mlp_forward(_ptr(p), f, h, _ptr(xx), xx.shape[0], _ptr(y)))
    return y


def mlp_grad(params, x, t, f: int = COST_FEATURES, h: int = MLP_HIDDEN):
    p, xx, tt = _f32(params), _f32(x).reshape(-1, f), _f32(t)
    g = np.empty(p.size, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(_lib.qs_mlp_grad(_ptr(p), f, h, _ptr(xx), _ptr(tt), xx.shape[0], _ptr(loss), _ptr(g)))
    return float(loss[0]), g


def mlp_train(params, x, t, steps: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
              f: int = COST_FEATURES, h: int = MLP_HIDDEN):
    """Adam on the GPU; returns (new params, last minibatch loss)."""
    p, xx, tt = _f32(params).copy(), _f32(x).reshape(-1, f), _f32(t)
    loss = np.zeros(1, dtype=np.float32)
    _check(_lib.qs_mlp_train(_ptr(p), f, h, _ptr(xx), _ptr(tt), xx.shape[0], steps, batch, lr, seed,
                             _ptr(loss)))
    return p, float(loss[0])


def mlp_init(seed: int, f: int = COST_FEATURES, h: int = MLP_HIDDEN) -> np.ndarray:
    """He-style random initial parameters (biases zero)."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((h, f)) * np.sqrt(2.0 / f)
    w2 = rng.standard_normal((h, h)) * np.sqrt(2.0 / h)
    w3 = rng.standard_normal(h) * np.sqrt(1.0 / h)
    return np.concatenate([w1.ravel(), np.zeros(h), w2.ravel(), np.zeros(h), w3, np.zeros(1)]).astype(
        np.float32)


def cost_model_set(params) -> None:
    if params is None:
        _check(_lib.qs_cost_model_set(None, COST_FEATURES, MLP_HIDDEN))
        return
    p = _f32(params)
    _check(_lib.qs_cost_model_set(_ptr(p), COST_FEATURES, MLP_HIDDEN))


class Circuit:
    """qs_circuit built from generator objects (Gate / Noise / Marker)."""

    def __init__(self, ops: Iterable = ()):
        h = C.c_void_p()
        _check(_lib.qs_circuit_create(C.byref(h)))
        self._h = h
        for o in ops:
            self.append(o)

    @property
    def handle(self):
        return self._h

    def append(self, o) -> None:
        k = o.kind
        if k == "gate":
            t, c, m = _ints(o.targets), _ints(o.controls), _mat(o.matrix)
            _check(_lib.qs_circuit_append_gate(self._h, _ptr(t), len(t), _ptr(c), len(c), _ptr(m)))
        elif k == "noise":
            t, kr = _ints(o.targets), _mat(o.kraus)
            _check(_lib.qs_circuit_append_noise(self._h, _ptr(t), len(t), _ptr(kr),
                                                int(np.asarray(o.kraus).shape[0])))
        elif k == "dagger":
            _check(_lib.qs_circuit_begin_dagger(self._h))
        elif k == "enddagger":
            _check(_lib.qs_circuit_end_dagger(self._h))
        elif k == "control":
            _check(_lib.qs_circuit_begin_control(self._h, int(o.qubit)))
        elif k == "endcontrol":
            _check(_lib.qs_circuit_end_control(self._h))
        else:
            raise ValueError("unknown op kind %r" % k)

    def plan_info(self, n: int, dtype: int = C64, plan: int = PLAN_GREEDY, k_max: int = 0,
                  tile_qubits: int = 0):
        o = RunOpts(plan=plan, k_max=k_max, tile_qubits=tile_qubits)
        sw, bl, lg = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.qs_circuit_plan_info(self._h, n, dtype, C.byref(o), C.byref(sw), C.byref(bl),
                                         C.byref(lg)))
        return {"sweeps": sw.value, "blocks": bl.value, "gates": lg.value}

    def partial_cuts(self, n: int, part_a: int) -> int:
        """qs_partial_cuts: gates cut at the dividing line between the qubits of
        the mask part_a and the rest."""
        c = C.c_int()
        _check(_lib.qs_partial_cuts(self._h, n, part_a, C.byref(c)))
        return c.value

    def partial_amplitudes(self, n: int, part_a: int, idx, dtype: int = C128, plan: int = PLAN_UNFUSED,
                           k_max: int = 0, tile_qubits: int = 0):
        """qs_partial_amplitudes: (complex128 amplitudes at idx, number of cuts)."""
        ix = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
        out = np.empty(ix.size, dtype=np.complex128)
        o = RunOpts(plan=plan, k_max=k_max, tile_qubits=tile_qubits)
        c = C.c_int()
        _check(_lib.qs_partial_amplitudes(self._h, n, dtype, part_a, _ptr(ix), ix.size,
                                          _ptr(out.view(np.float64)), C.byref(o), C.byref(c)))
        return out, c.value

    def single_amplitudes(self, n: int, bits, nslice: int = 0):
        """qs_single_amplitudes: (complex128 amplitudes <x|C|0...0> for each
        bitstring x in `bits`, shape of the contraction as a dict)."""
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64).reshape(-1))
        out = np.empty(b.size, dtype=np.complex128)
        info = SingleInfo()
        _check(_lib.qs_single_amplitudes(self._h, n, _ptr(b), b.size, nslice, _ptr(out.view(np.float64)),
                                         C.byref(info)))
        return out, {f: getattr(info, f) for f, _ in SingleInfo._fields_}

    def single_plan(self, n: int, nslice: int = 0) -> dict:
        """qs_single_plan: the contraction's shape for one bitstring (host only)."""
        info = SingleInfo()
        _check(_lib.qs_single_plan(self._h, n, nslice, C.byref(info)))
        return {f: getattr(info, f) for f, _ in SingleInfo._fields_}

    def autotune_result(self, n: int, dtype: int = C64):
        """(tried, candidates, tile_qubits, k_max, seconds) of QS_PLAN_AUTOTUNE
        for states of this shape."""
        tr, nc, tq, km, sec = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_double()
        _check(_lib.qs_circuit_autotune_result(self._h, n, dtype, C.byref(tr), C.byref(nc), C.byref(tq),
                                               C.byref(km), C.byref(sec)))
        return tr.value, nc.value, tq.value, km.value, sec.value

    def counts(self):
        g, z, l = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.qs_circuit_counts(self._h, C.byref(g), C.byref(z), C.byref(l)))
        return g.value, z.value, l.value

    def close(self):
        if self._h:
            _lib.qs_circuit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _info_dict(info: ScriptInfo) -> dict:
    return {"n": info.n, "creg": info.creg, "measures": info.measures,
            "pmeasure": [info.pmeasure[k] for k in range(info.pmeasure_n)]}


def script_parse(text: str):
    """qs_script_parse: (Circuit, info) for an App. A-1 script."""
    h, info = C.c_void_p(), ScriptInfo()
    _check(_lib.qs_script_parse(text.encode(), C.byref(h), C.byref(info)))
    c = Circuit.__new__(Circuit)
    c._h = h
    return c, _info_dict(info)


def script_run(text: str, dtype: int = C128, seed: int = 0, plan: int = PLAN_UNFUSED):
    """qs_script_run: (classical registers, PMEASURE probabilities, info)."""
    h, info = C.c_void_p(), ScriptInfo()
    _check(_lib.qs_script_parse(text.encode(), C.byref(h), C.byref(info)))
    _lib.qs_circuit_destroy(h)
    creg = (C.c_int * max(info.creg, 1))()
    probs = np.zeros(1 << info.pmeasure_n if info.pmeasure_n else 1)
    _check(_lib.qs_script_run(text.encode(), dtype, seed, plan, creg, info.creg, _ptr(probs), probs.size,
                              C.byref(info)))
    return ([creg[j] for j in range(info.creg)], probs if info.pmeasure_n else None, _info_dict(info))


def probabilities_noalloc(device_amps: int, n: int, dtype: int, qubits, device_out: int, stream: int = 0):
    """qs_probabilities_noalloc on raw device pointers (ints): enqueues the
    reduction on `stream` and returns at once; nothing is allocated."""
    q = None if qubits is None else _ints(qubits)
    _check(_lib.qs_probabilities_noalloc(C.c_void_p(device_amps), n, dtype, _ptr(q), 0 if q is None else len(q),
                                         C.c_void_p(device_out), C.c_void_p(stream or 0)))


class State:
    """A 2^n-amplitude state on the current HIP device (qs_state)."""

    def __init__(self, n: int, dtype: int = C128, buffer=None, stream=None):
        h = C.c_void_p()
        self._keep = None
        if buffer is None:
            _check(_lib.qs_create(n, dtype, C.byref(h)))
        else:
            # torch tensor (or anything exposing data_ptr / nbytes) as borrowed storage
            ptr = buffer.data_ptr()
            nbytes = buffer.numel() * buffer.element_size()
            self._keep = buffer
            _check(_lib.qs_create_from_buffer(n, dtype, C.c_void_p(ptr), nbytes,
                                              C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self.n = n
        self.dtype = dtype

    @property
    def handle(self):
        return self._h

    def reset(self):
        _check(_lib.qs_reset(self._h))

    def set_amplitudes(self, psi: np.ndarray):
        a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
        assert a.size == 1 << self.n
        _check(_lib.qs_set_amplitudes(self._h, _ptr(a.view(np.float64))))

    def synchronize(self):
        _check(_lib.qs_synchronize(self._h))

    def apply_gate(self, targets: Sequence[int], controls: Sequence[int], matrix) -> None:
        t, c, m = _ints(targets), _ints(controls), _mat(matrix)
        _check(_lib.qs_apply_gate(self._h, _ptr(t), len(t), _ptr(c), len(c), _ptr(m)))

    def apply_noisy_gate(self, targets, matrix, kraus, u: float, controls=()):
        t, c, m, kr = _ints(targets), _ints(controls), _mat(matrix), _mat(kraus)
        ch, pc = C.c_int(), C.c_double()
        _check(_lib.qs_apply_noisy_gate(self._h, _ptr(t), len(t), _ptr(c), len(c), _ptr(m),
                                        _ptr(kr), int(np.asarray(kraus).shape[0]), u,
                                        C.byref(ch), C.byref(pc)))
        return ch.value, pc.value

    def run(self, circuit: Circuit, plan: int = PLAN_UNFUSED, k_max: int = 0, seed: int = 0,
            traj: int = 0, nsites: int = 0, tile_qubits: int = 0, tile_order: int = 0):
        o = RunOpts(plan=plan, k_max=k_max, seed=seed, traj=traj, tile_qubits=tile_qubits,
                    tile_order=tile_order)
        chosen = None
        if nsites:
            chosen = (C.c_int64 * nsites)()
            o.chosen = chosen
            o.chosen_len = nsites
        _check(_lib.qs_run_circuit(self._h, circuit.handle, C.byref(o)))
        return np.array(chosen[:], dtype=np.int64) if chosen is not None else None

    def remap_pack(self, lq: Sequence[int], buffer) -> None:
        """qs_remap_pack into `buffer` (device memory exposing data_ptr(), e.g. a
        torch tensor of 2^n amplitudes of the state's dtype)."""
        q = _ints(lq)
        _check(_lib.qs_remap_pack(self._h, len(q), _ptr(q), C.c_void_p(buffer.data_ptr())))

    def remap_unpack(self, lq: Sequence[int], buffer) -> None:
        """qs_remap_unpack from `buffer` (as remap_pack)."""
        q = _ints(lq)
        _check(_lib.qs_remap_unpack(self._h, len(q), _ptr(q), C.c_void_p(buffer.data_ptr())))

    def amplitudes(self, idx: Optional[np.ndarray] = None) -> np.ndarray:
        if idx is None:
            out = np.empty(1 << self.n, dtype=np.complex128)
            _check(_lib.qs_amplitudes(self._h, None, out.size, _ptr(out.view(np.float64))))
            return out
        ix = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
        out = np.empty(ix.size, dtype=np.complex128)
        _check(_lib.qs_amplitudes(self._h, _ptr(ix), ix.size, _ptr(out.view(np.float64))))
        return out

    def probabilities(self, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
        if qubits is None:
            out = np.empty(1 << self.n, dtype=np.float64)
            _check(_lib.qs_probabilities(self._h, None, 0, _ptr(out)))
            return out
        q = _ints(qubits)
        out = np.empty(1 << len(q), dtype=np.float64)
        _check(_lib.qs_probabilities(self._h, _ptr(q), len(q), _ptr(out)))
        return out

    def norm(self) -> float:
        v = C.c_double()
        _check(_lib.qs_norm(self._h, C.byref(v)))
        return v.value

    def expect_z(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        _check(_lib.qs_expect_z(self._h, _ptr(out)))
        return out

    def profile(self, on: bool = True):
        _check(_lib.qs_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        _check(_lib.qs_profile_reset(self._h))

    def profile_query(self, kernel: int):
        l, ms, b, f = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        _check(_lib.qs_profile_query(self._h, kernel, C.byref(l), C.byref(ms), C.byref(b),
                                     C.byref(f)))
        return {"launches": l.value, "ms": ms.value, "bytes": b.value, "flops": f.value}

    def profile_samples(self, capacity: int = 100000):
        """(features [count, 16], ln ns per amplitude [count]) of the profiled tile sweeps."""
        f = np.empty((capacity, COST_FEATURES), dtype=np.float32)
        y = np.empty(capacity, dtype=np.float32)
        cnt = C.c_int64()
        _check(_lib.qs_profile_samples(self._h, _ptr(f), _ptr(y), capacity, C.byref(cnt)))
        return f[: cnt.value].copy(), y[: cnt.value].copy()

    def info(self):
        n, dt = C.c_int(), C.c_int()
        dev, st = C.c_void_p(), C.c_void_p()
        _check(_lib.qs_info(self._h, C.byref(n), C.byref(dt), C.byref(dev), C.byref(st)))
        return {"n": n.value, "dtype": dt.value, "device_ptr": dev.value, "stream": st.value}

    def close(self):
        if self._h:
            _lib.qs_destroy(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_trajectories(circuits: Sequence[Circuit], widths: Sequence[int], dtype: int = C64,
                     seed: int = 0, plan: int = PLAN_GREEDY, k_max: int = 0, tile_qubits: int = 0,
                     direct_launch: bool = False):
    """qs_run_trajectories: (z [sum widths], statistics of the call as a dict,
    including traj_per_s)."""
    arr = (C.c_void_p * len(circuits))(*[c.handle.value for c in circuits])
    w = _ints(widths)
    z = np.empty(int(w.sum()), dtype=np.float64)
    o = RunOpts(plan=plan, k_max=k_max, tile_qubits=tile_qubits, direct_launch=1 if direct_launch else 0)
    rate = C.c_double()
    _check(_lib.qs_run_trajectories(C.cast(arr, C.c_void_p), _ptr(w), len(circuits), dtype, seed,
                                    C.byref(o), _ptr(z), C.byref(rate)))
    st = TrajStats()
    _check(_lib.qs_trajectory_stats(C.byref(st)))
    info = {f: getattr(st, f) for f, _ in TrajStats._fields_}
    info["traj_per_s"] = rate.value
    return z, info
