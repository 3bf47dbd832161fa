"""Reader of the hand-worked fixtures under tests/golden/.

Each file holds one or more cases:

    case <name>
    dtype u8|f32
    input           rows of the [C][T] beam, one channel per line
    steps           one step per line: <td|fd> <k> <mean|median> <bin>
    output          the expected [C][T] result
    flags           the expected flag bytes (bit j: step j replaced the sample)
    end

float32 values are written as hexadecimal floating point.  Lines starting
with '#' carry the derivation and its citation.
"""
from __future__ import annotations

import glob
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _parse_value(tok: str, dtype: str):
    return float.fromhex(tok) if dtype == "f32" else int(tok)


def load_cases():
    """[(id, x, steps, out, flags)] for every case of every fixture."""
    cases = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))):
        name = os.path.splitext(os.path.basename(path))[0]
        cur, section = None, None
        for raw in open(path):
            line = raw.strip()
            if not line or line.startswith("#"):
                continue
            word = line.split()[0]
            if word == "case":
                cur = {"name": line[5:].strip(), "input": [], "steps": [], "output": [], "flags": []}
                section = None
            elif word == "dtype":
                cur["dtype"] = line.split()[1]
            elif word in ("input", "steps", "output", "flags"):
                section = word
            elif word == "end":
                dt = np.uint8 if cur["dtype"] == "u8" else np.float32
                conv = lambda rows, d=cur["dtype"]: [[_parse_value(t, d) for t in r] for r in rows]
                x = np.array(conv(cur["input"]), dtype=dt)
                out = np.array(conv(cur["output"]), dtype=dt)
                fl = np.array([[int(t) for t in r] for r in cur["flags"]], dtype=np.uint8)
                steps = [(s[0], float(s[1]), s[2], int(s[3])) for s in cur["steps"]]
                assert x.shape == out.shape == fl.shape, path
                cases.append((f"{name}: {cur['name']}", x, steps, out, fl))
                cur = None
            else:
                cur[section].append(line.split())
    return cases
