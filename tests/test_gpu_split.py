"""GPU parity: full products of fewer instances than CUs, whose bands run on
several work-groups per instance (carry words in a workspace, the closing
strip carry scan in a second launch), against the oracle on every instance
and against the bytes of one work-group per instance."""
import json

import numpy as np
import pytest

from gpu_util import dev, host, oracle_map, rand_limbs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bi():
    import paper_2607_28897_amd as m
    m.lib()
    yield m
    m.set_mfma_config(0, 0, 0)
    m.set_mfma_tile(0)
    m.autotune_load(None)


# (batch, na, nb): one 2^19-bit product, the largest operands, unequal
# operands, ragged strip counts, and batches up to a quarter of the CU count
CASES = [(1, 16384, 16384), (1, 18432, 18432), (2, 16384, 1000), (3, 5000, 5000), (7, 4096, 4100),
         (17, 4096, 4096), (60, 5000, 3500), (64, 4096, 4096), (64, 16384, 16384),
         (1, 16384, 1), (3, 2, 12000)]


@pytest.mark.parametrize("batch,na,nb", CASES)
def test_split_every_instance(bi, orc, batch, na, nb):
    g = np.random.default_rng(batch * 7 + na + nb)
    a = rand_limbs(g, batch, na)
    b = rand_limbs(g, batch, nb)
    a[0] = 0xFFFFFFFF                      # carries through whole strips
    b[0] = 0xFFFFFFFF
    if batch > 1 and nb > 1:
        b[1, 1:] = 0                       # a * small: long all-ones and zero runs
        b[1, 0] = 3
    assert bi.mfma_split_parts(na, nb, batch) >= 4
    p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
    want = oracle_map(lambda i: orc.mul1(a[i], b[i]), range(batch))
    bad = [i for i in range(batch) if not np.array_equal(p[i], want[i])]
    assert not bad, bad[:10]


@pytest.mark.parametrize("na,nb", [(16384, 16384), (3000, 5000)])
def test_split_equals_one_work_group_per_instance(bi, na, nb):
    """One instance alone (split) and the same instance among 256 (a whole
    work-group each), and alone with a configuration forced (no split): the
    same bytes."""
    import torch
    g = np.random.default_rng(na)
    a = rand_limbs(g, 1, na)
    b = rand_limbs(g, 1, nb)
    ta, tb = dev(a), dev(b)
    assert bi.mfma_split_parts(na, nb, 1) >= 4
    alone = host(bi.mul(ta, tb, bi.MUL_MFMA))[0]
    assert bi.mfma_split_parts(na, nb, 256) == 1
    many = host(bi.mul(ta.expand(256, -1).contiguous(), tb.expand(256, -1).contiguous(),
                       bi.MUL_MFMA))
    assert all(np.array_equal(alone, many[i]) for i in (0, 97, 255))
    P, w, d = bi.mfma_config(na, nb)
    bi.set_mfma_config(P, 0, 0)
    try:
        assert bi.mfma_split_parts(na, nb, 1) == 1
        forced = host(bi.mul(ta, tb, bi.MUL_MFMA))[0]
    finally:
        bi.set_mfma_config(0, 0, 0)
    assert np.array_equal(alone, forced)
    torch.cuda.synchronize()


def test_split_seven_bit_digits_from_table(bi, orc, tmp_path):
    # a loaded table (not a forced configuration) with 7-bit digits: the
    # split runs 7-bit strips of 56 limbs
    path = str(tmp_path / "t7.json")
    json.dump({"bins": [{"max_limbs": 18432, "strips_per_band": 16, "waves": 8, "digit_bits": 7}]},
              open(path, "w"))
    bi.autotune_load(path)
    try:
        g = np.random.default_rng(77)
        for batch, n in ((1, 16000), (5, 5000)):
            a = rand_limbs(g, batch, n)
            b = rand_limbs(g, batch, n)
            assert bi.mfma_config(n, n)[2] == 7 and bi.mfma_split_parts(n, n, batch) >= 4
            p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
            for i in range(batch):
                assert np.array_equal(p[i], orc.mul1(a[i], b[i])), (batch, n, i)
    finally:
        bi.autotune_load(None)


def test_split_parts_query(bi):
    # no split for full batches, small products, or a forced configuration
    assert bi.mfma_split_parts(16384, 16384, 256) == 1
    assert bi.mfma_split_parts(16384, 16384, 1000) == 1
    assert bi.mfma_split_parts(300, 300, 1) == 1
    assert bi.mfma_split_parts(16384, 16384, 1) == 32     # 128 bands of 4 strips, four per part
    assert bi.mfma_split_parts(16384, 16384, 64) == 4     # the CUs once
    assert bi.mfma_split_parts(16384, 16384, 128) == 1    # two parts: not split
    assert bi.mfma_split_parts(1024, 1024, 64) == 1
    assert bi.mfma_split_parts(2048, 2048, 1) == 1         # 64 strips: too few bands
    bi.set_mfma_config(0, 4, 0)
    try:
        assert bi.mfma_split_parts(16384, 16384, 1) == 1
    finally:
        bi.set_mfma_config(0, 0, 0)


@pytest.mark.parametrize("batch,n", [(1, 16384), (1, 18432), (3, 9000), (16, 8192), (64, 16384)])
def test_split_products_mod_b_n(bi, orc, batch, n):
    """bigint_mullo (a b mod B^n) on the split path: only the strips below
    limb n, every instance against the oracle and against the bytes of one
    work-group per instance (configuration forced)."""
    g = np.random.default_rng(batch + n)
    a = rand_limbs(g, batch, n)
    b = rand_limbs(g, batch, n)
    a[0] = 0xFFFFFFFF
    b[0] = 0xFFFFFFFF                    # (B^n - 1)^2 mod B^n = 1
    p = host(bi.mullo(dev(a), dev(b)))
    want = oracle_map(lambda i: orc.mullo1(a[i], b[i]), range(batch))
    assert all(np.array_equal(p[i], want[i]) for i in range(batch))
    P, w, d = bi.mfma_config(n, n)
    bi.set_mfma_config(P, 0, 0)
    try:
        forced = host(bi.mullo(dev(a), dev(b)))
    finally:
        bi.set_mfma_config(0, 0, 0)
    assert np.array_equal(p, forced)
