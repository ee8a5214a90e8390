"""Golden worked examples (tests/golden/cases.json, written by the oracle via
tests/golden/make_golden.py): the stored values are checked against their
closed forms with Python integers, and the GPU against the stored values."""
import json
import os

import numpy as np
import pytest

from conftest import to_int

B = 2**32
HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "cases.json")))


def limbs(h):
    return np.array([int(x, 16) for x in h], np.uint32)


def test_closed_forms():
    ops = {c["op"] for c in CASES}
    assert {"add", "sub", "mul", "divmod", "shinv", "conv7"} <= ops
    for c in CASES:
        if c["op"] == "add":
            a, b = to_int(limbs(c["a"])), to_int(limbs(c["b"]))
            assert a + b == B**5 and to_int(limbs(c["r"])) == 0 and c["carry"] == 1
        elif c["op"] == "sub":
            assert to_int(limbs(c["r"])) == B**5 - 1 and c["carry"] == 1
        elif c["op"] == "mul":
            a, b = to_int(limbs(c["a"])), to_int(limbs(c["b"]))
            r = to_int(limbs(c["r"]))
            if len(c["a"]) == 3 and len(c["b"]) == 3:
                assert r == (B**3 - 1) ** 2
            else:
                assert r == 15 + 22 * B + 13 * B**2 + 4 * B**3
            assert r == a * b
        elif c["op"] == "divmod":
            assert to_int(limbs(c["q"])) == B**2 + 1 and to_int(limbs(c["r"])) == 0
        elif c["op"] == "shinv":
            assert to_int(limbs(c["w"])) == B**2 - B
        elif c["op"] == "conv7":
            assert c["digits"] == [127, 127, 127, 127, 15]
            assert c["c"] == [int(x) for x in np.convolve(c["digits"], c["digits"])]


@pytest.mark.gpu
def test_gpu_matches_golden():
    from gpu_util import dev, host
    import paper_2607_28897_amd as bi
    for c in CASES:
        if c["op"] == "add":
            r, cy = bi.add(dev(limbs(c["a"])[None]), dev(limbs(c["b"])[None]))
            assert np.array_equal(host(r)[0], limbs(c["r"])) and int(host(cy)[0]) == c["carry"]
        elif c["op"] == "sub":
            r, cy = bi.sub(dev(limbs(c["a"])[None]), dev(limbs(c["b"])[None]))
            assert np.array_equal(host(r)[0], limbs(c["r"])) and int(host(cy)[0]) == c["carry"]
        elif c["op"] == "mul":
            for algo in (bi.MUL_PLAIN, bi.MUL_MFMA):
                r = bi.mul(dev(limbs(c["a"])[None]), dev(limbs(c["b"])[None]), algo)
                assert np.array_equal(host(r)[0], limbs(c["r"]))
        elif c["op"] == "divmod":
            q, r, st = bi.divmod(dev(limbs(c["a"])[None]), dev(limbs(c["b"])[None]))
            assert np.array_equal(host(q)[0], limbs(c["q"])) and np.array_equal(host(r)[0], limbs(c["r"]))
        elif c["op"] == "shinv":
            w = bi.shinv(dev(limbs(c["b"])[None]), c["h"])
            assert np.array_equal(host(w)[0], limbs(c["w"]))
        elif c["op"] == "conv7":
            a = dev(limbs(c["a"])[None])
            assert bi.digits7(a).cpu().numpy()[0].tolist() == c["digits"]
            assert bi.conv7(a, a).cpu().numpy()[0].tolist() == c["c"]
