"""Writes tests/golden/cases.json from the CPU oracle only.

Each case is a small worked example whose value also has a closed form or a
hand-checkable definition; tests/test_golden.py checks the stored values
against those closed forms (Python integers) and the GPU against the stored
values.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402


def hexlimbs(a):
    return [f"{int(x):08x}" for x in np.asarray(a, np.uint32)]


def main():
    oracle.build()
    B = 2**32
    cases = []
    # Section 5.1: a carry that ripples through every limb, (B^5 - 1) + 1 = B^5
    a = np.full(5, 0xFFFFFFFF, np.uint32)
    b = np.array([1, 0, 0, 0, 0], np.uint32)
    r, c = oracle.add1(a, b)
    cases.append({"op": "add", "cite": "Section 5.1 (carry propagation scan)", "a": hexlimbs(a),
                  "b": hexlimbs(b), "r": hexlimbs(r), "carry": c, "closed_form": "(B^5-1)+1 = B^5"})
    # mirror for subtraction: 0 - 1 = B^5 - 1 with a borrow
    z = np.zeros(5, np.uint32)
    r, c = oracle.sub1(z, b)
    cases.append({"op": "sub", "cite": "Section 5.3 (bsubReg' in step)", "a": hexlimbs(z),
                  "b": hexlimbs(b), "r": hexlimbs(r), "carry": c, "closed_form": "0-1 = B^5-1, borrow 1"})
    # Section 5.2: (B^3 - 1)^2 = B^6 - 2 B^3 + 1
    o = np.full(3, 0xFFFFFFFF, np.uint32)
    cases.append({"op": "mul", "cite": "Section 5.2 (quadratic product)", "a": hexlimbs(o),
                  "b": hexlimbs(o), "r": hexlimbs(oracle.mul1(o, o)), "closed_form": "(B^3-1)^2"})
    # a small hand-checkable product: (3 + 2B + B^2)(5 + 4B) = 15 + 22B + 13B^2 + 4B^3
    x = np.array([3, 2, 1], np.uint32)
    y = np.array([5, 4], np.uint32)
    cases.append({"op": "mul", "cite": "Section 5.2 (C_k = sum A_i B_j)", "a": hexlimbs(x),
                  "b": hexlimbs(y), "r": hexlimbs(oracle.mul1(x, y)),
                  "closed_form": "15 + 22B + 13B^2 + 4B^3"})
    # Section 5.3: (B^4 - 1) / (B^2 - 1) = B^2 + 1 remainder 0
    u = np.full(4, 0xFFFFFFFF, np.uint32)
    v = np.full(2, 0xFFFFFFFF, np.uint32)
    q, rr, st = oracle.divmod1(u, v)
    cases.append({"op": "divmod", "cite": "Section 5.3 (quotient and remainder)", "a": hexlimbs(u),
                  "b": hexlimbs(v), "q": hexlimbs(q), "r": hexlimbs(rr), "status": st,
                  "closed_form": "(B^4-1)/(B^2-1) = B^2+1 rem 0"})
    # shifted inverse floor(B^3 / (B + 1)) = B^2 - B + 1 - 1 = B^2 - B (since B^3 = (B+1)(B^2-B+1) - 1)
    w, st = oracle.shinv1(np.array([1, 1], np.uint32), 3)
    cases.append({"op": "shinv", "cite": "Section 5.3 (whole shifted inverse)", "b": ["00000001", "00000001"],
                  "h": 3, "w": hexlimbs(w), "closed_form": "floor(B^3/(B+1)) = B^2 - B"})
    # 7-bit digits of one all-ones limb and their self-convolution
    d = oracle.digits1(np.array([0xFFFFFFFF], np.uint32), 7)
    cases.append({"op": "conv7", "cite": "Section 5.2 formula over 7-bit digits", "a": ["ffffffff"],
                  "digits": [int(t) for t in d], "c": [int(t) for t in oracle.conv1(d, d)],
                  "closed_form": "digits 127,127,127,127,15"})
    with open(os.path.join(HERE, "cases.json"), "w") as f:
        json.dump(cases, f, indent=1)
    print(f"wrote {len(cases)} cases")


if __name__ == "__main__":
    main()
