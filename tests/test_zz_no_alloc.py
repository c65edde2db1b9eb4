"""qs_probabilities_noalloc (the entry point for callers that cannot
allocate) against qs_probabilities on the same states: calls in a row, each
after the first on a smaller state or fewer qubits, every result to the FP64
reduction bound of the parity tests (1e-13; the kernels are the same, but
binned sums of more than eight outcomes accumulate with atomics in LDS, so
their last bits depend on the order).  Device memory for the results is the
amplitude buffer of another state (a complex128 state of nq - 1 qubits holds
2^nq doubles), read back through qs_amplitudes."""
import numpy as np
import pytest

from paper_2008_07140_amd import circuits as cg

pytestmark = pytest.mark.gpu


def _state(qs, n, dtype, seed):
    rows = n // 4 if n % 4 == 0 else 2
    s = qs.State(n, dtype)
    s.run(qs.Circuit(cg.random_circuit(rows, n // rows, 6, seed=seed, cu3_prob=0.1)))
    s.synchronize()
    return s


def _device_doubles(qs, nq):
    """A device buffer of 2^nq doubles (nq >= 1) owned by a state."""
    return qs.State(nq - 1, qs.C128)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_probabilities_match_the_allocating_call(dtype):
    from paper_2008_07140_amd import qs
    dt = qs.C128 if dtype == "c128" else qs.C64
    cases = [(20, [19, 3, 0, 7, 11]), (14, [2, 13]), (16, None), (12, list(range(11, -1, -1))),
             (18, [5, 1, 17, 9, 12, 3, 0, 14, 8, 2, 11, 16])]
    for k, (n, qubits) in enumerate(cases):
        print("[noalloc] %s n=%d qubits=%s" % (dtype, n, qubits), flush=True)
        s = _state(qs, n, dt, 2100 + k)
        info = s.info()
        nq = n if qubits is None else len(qubits)
        out = _device_doubles(qs, nq)
        qs.probabilities_noalloc(info["device_ptr"], n, dt, qubits, out.info()["device_ptr"], info["stream"])
        s.synchronize()
        got = out.amplitudes().view(np.float64)
        want = s.probabilities(qubits)
        assert got.size == want.size
        assert np.max(np.abs(got - want)) <= 1e-13
        assert abs(got.sum() - s.norm()) <= 1e-12
        out.close()
        s.close()


def test_noalloc_rejects_bad_arguments_before_any_work():
    from paper_2008_07140_amd import qs
    out = _device_doubles(qs, 3)
    amp = qs.State(4, qs.C128)
    o, a = out.info()["device_ptr"], amp.info()["device_ptr"]
    for args, st in (((0, 4, qs.C128, [0], o), -1), ((a, 0, qs.C128, [0], o), -1),
                     ((a, 4, qs.C128, [0, 0], o), -2), ((a, 4, qs.C128, [4], o), -2),
                     ((a + 8, 4, qs.C128, [0], o), -1), ((a, 4, 9, [0], o), -1)):
        with pytest.raises(qs.QSError) as e:
            qs.probabilities_noalloc(*args)
        assert e.value.status == st
    out.close()
    amp.close()
