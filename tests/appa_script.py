"""Minimal reader for the App. A-1 instruction syntax, used by the tests.

Only what the worked example and the tests need: QINIT, CREG (ignored),
H/X/Y/Z/S/T, RX/RY/RZ, U4, CNOT/CZ/CR, SWAP/ISWAP, TOFFOLI,
DAGGER/ENDDAGGER, CONTROL/ENDCONTROL and PMEASURE.  Matrices come from a
caller-supplied ``named_gate(name, params)`` so the same script can be fed to
different gate tables.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Tuple

import numpy as np


@dataclass
class SGate:
    targets: Tuple[int, ...]
    controls: Tuple[int, ...]
    matrix: np.ndarray
    name: str = ""
    kind: str = field(default="gate", init=False)


@dataclass
class SMarker:
    kind: str
    qubit: int = -1


def _angle(tok: str) -> float:
    tok = tok.strip().strip('"').strip()
    return float(eval(tok, {"__builtins__": {}}, {"pi": math.pi}))


def parse(text: str, named_gate: Callable[[str, tuple], np.ndarray]):
    """Returns (n, ops, pmeasure_qubits, printed_output or None)."""
    n = None
    ops: List = []
    pm = None
    out = {}
    section = None
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        if line.startswith("%"):
            section = line[1:].strip().lower()
            continue
        if section == "output":
            k, v = line.split(":")
            out[k.strip()] = float(v)
            continue
        head, _, rest = line.partition(" ")
        head = head.upper()
        args = [a.strip() for a in rest.split(",")] if rest.strip() else []
        if head == "QINIT":
            n = int(args[0])
        elif head == "CREG":
            pass
        elif head in ("H", "X", "Y", "Z", "S", "T"):
            ops.append(SGate((int(args[0]),), (), named_gate(head, ()), head))
        elif head in ("RX", "RY", "RZ"):
            ops.append(SGate((int(args[0]),), (), named_gate(head, (_angle(args[1]),)), head))
        elif head == "U4":
            vals = tuple(_angle(a) for a in args[1:])
            ops.append(SGate((int(args[0]),), (), named_gate("U4", vals), head))
        elif head in ("CNOT", "CZ", "SWAP", "ISWAP"):
            ops.append(SGate((int(args[0]), int(args[1])), (), named_gate(head, ()), head))
        elif head == "CR":
            ops.append(SGate((int(args[0]), int(args[1])), (),
                             named_gate("CR", (_angle(args[2]),)), head))
        elif head == "TOFFOLI":
            ops.append(SGate(tuple(int(a) for a in args[:3]), (), named_gate(head, ()), head))
        elif head == "DAGGER":
            ops.append(SMarker("dagger"))
        elif head == "ENDDAGGER":
            ops.append(SMarker("enddagger"))
        elif head == "CONTROL":
            ops.append(SMarker("control", int(args[0])))
        elif head == "ENDCONTROL":
            ops.append(SMarker("endcontrol"))
        elif head == "PMEASURE":
            pm = [int(a) for a in args]
        else:
            raise ValueError("unknown instruction %r" % head)
    printed = None
    if out:
        printed = np.array([out[k] for k in sorted(out, key=lambda s: int(s, 2))])
    return n, ops, pm, printed
