"""GPU parity: plain u64 multiply and MFMA-split multiply against the oracle,
bit for bit, through the C-ABI; plus the intermediate steps of the MFMA path
(digit split, int32 coefficients) and tile-configuration invariance."""
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


# the plain kernel, and the MFMA-split kernel with 7-bit and offset 8-bit
# digits on 16x16x64 tiles, and with 8-bit digits on 32x32x32 tiles
ALGOS = ["plain", "mfma7", "mfma8", "mfma8t32"]


def _mul(bi, ta, tb, name):
    if name == "plain":
        return bi.mul(ta, tb, bi.MUL_PLAIN)
    bi.set_mfma_config(0, 0, 7 if name == "mfma7" else 8)
    bi.set_mfma_tile(32 if name == "mfma8t32" else 16)
    try:
        return bi.mul(ta, tb, bi.MUL_MFMA)
    finally:
        bi.set_mfma_config(0, 0, 0)
        bi.set_mfma_tile(0)


# ---- the steps of the MFMA path ---------------------------------------------------

@pytest.mark.parametrize("n", [1, 7, 8, 100, 1024, 4097])
def test_digit_split(bi, orc, n):
    g = np.random.default_rng(n)
    a = rand_limbs(g, 3, n)
    d = bi.digits7(dev(a)).cpu().numpy()
    for i in range(3):
        assert np.array_equal(d[i], orc.digits1(a[i], 7))


@pytest.mark.parametrize("na,nb", [(1, 1), (2, 1), (7, 7), (8, 9), (56, 56), (63, 65), (100, 300),
                                   (448, 448), (449, 447), (1024, 1024), (2000, 1500)])
def test_coefficients(bi, orc, na, nb):
    g = np.random.default_rng(na * 1000 + nb)
    a = rand_limbs(g, 2, na)
    b = rand_limbs(g, 2, nb)
    c = bi.conv7(dev(a), dev(b)).cpu().numpy()
    for i in range(2):
        want = orc.conv1(orc.digits1(a[i]), orc.digits1(b[i]))
        assert np.array_equal(c[i].astype(np.int64), want)


def test_coefficients_all_ones_bound(bi, orc):
    n = 4096
    a = np.full((1, n), 0xFFFFFFFF, np.uint32)
    c = bi.conv7(dev(a), dev(a)).cpu().numpy()[0]
    want = orc.conv1(orc.digits1(a[0]), orc.digits1(a[0]))
    assert np.array_equal(c.astype(np.int64), want)


# ---- full products --------------------------------------------------------------------

@pytest.mark.parametrize("algo", ALGOS)
def test_pairs_2e15(bi, orc, algo):
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e15()
    p = _mul(bi, dev(c["a"]), dev(c["b"]), algo)
    assert np.array_equal(host(p), orc.mul(c["a"], c["b"]))


@pytest.fixture(scope="module")
def pairs_2e17(orc):
    """1024 pairs of 2^17-bit integers (half carry-adversarial) and the
    oracle's product of every pair."""
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e17_mixed()
    c["want"] = np.stack(oracle_map(lambda i: orc.mul1(c["a"][i], c["b"][i]), range(1024)))
    return c


@pytest.fixture(scope="module")
def pairs_2e19(orc):
    """256 pairs of 2^19-bit integers and the oracle's product of every pair."""
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e19()
    c["want"] = np.stack(oracle_map(lambda i: orc.mul1(c["a"][i], c["b"][i]), range(256)))
    return c


def _rows_differing(got, want):
    return [int(i) for i in np.nonzero((got != want).any(axis=1))[0]]


@pytest.mark.parametrize("algo", ALGOS)
def test_pairs_2e17_every_instance(bi, pairs_2e17, algo):
    """All 1024 products of the 2^17-bit configuration, uniform and
    carry-adversarial halves, against the oracle limb by limb."""
    c = pairs_2e17
    p = host(_mul(bi, dev(c["a"]), dev(c["b"]), algo))
    assert p.shape == c["want"].shape
    assert _rows_differing(p, c["want"]) == []


@pytest.mark.parametrize("algo", ALGOS + ["karatsuba"])
def test_pairs_2e19_every_instance(bi, pairs_2e19, algo):
    """All 256 products of the 2^19-bit configuration (the headline), for the
    plain kernel, both digit widths of the MFMA-split kernel and one
    Karatsuba level, against the oracle limb by limb."""
    c = pairs_2e19
    if algo == "karatsuba":
        p = host(bi.mul(dev(c["a"]), dev(c["b"]), bi.MUL_KARATSUBA))
    else:
        p = host(_mul(bi, dev(c["a"]), dev(c["b"]), algo))
    assert _rows_differing(p, c["want"]) == []


@pytest.mark.parametrize("algo", ALGOS)
def test_all_ones_2e19(bi, orc, algo):
    # (B^n - 1)^2: every 7-bit digit is 127, the largest coefficients possible
    n = 16384
    a = np.full((1, n), 0xFFFFFFFF, np.uint32)
    p = host(_mul(bi, dev(a), dev(a), algo))[0]
    want = np.concatenate([[1], np.zeros(n - 1), [0xFFFFFFFE], np.full(n - 1, 0xFFFFFFFF)]).astype(np.uint32)
    assert np.array_equal(p, want)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("na,nb", [(1, 1), (1, 2), (3, 1), (5, 5), (55, 57), (64, 64), (111, 1000),
                                   (1000, 111), (2047, 2049), (4096, 1), (8191, 8193)])
def test_shapes(bi, orc, algo, na, nb):
    g = np.random.default_rng(na * 7 + nb)
    a = rand_limbs(g, 3, na)
    b = rand_limbs(g, 3, nb)
    b[2] = 0xFFFFFFFF
    p = host(_mul(bi, dev(a), dev(b), algo))
    for i in range(3):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i])), i


def test_zero_and_one(bi, orc):
    g = np.random.default_rng(1)
    n = 3000
    a = rand_limbs(g, 2, n)
    b = np.zeros((2, n), np.uint32)
    b[1, 0] = 1
    for algo in ALGOS:
        p = host(_mul(bi, dev(a), dev(b), algo))
        assert not p[0].any()
        assert np.array_equal(p[1][:n], a[1]) and not p[1][n:].any()


@pytest.mark.parametrize("dw", [7, 8])
@pytest.mark.parametrize("P,waves", [(4, 4), (4, 8), (8, 4), (8, 8), (16, 4), (16, 8)])
def test_tile_configs_identical(bi, orc, P, waves, dw):
    g = np.random.default_rng(P * 10 + waves)
    a = rand_limbs(g, 2, 3333)
    b = rand_limbs(g, 2, 2900)
    bi.set_mfma_config(P, waves, dw)
    try:
        p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
    finally:
        bi.set_mfma_config(0, 0, 0)
    for i in range(2):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i]))


def test_plain_matches_mfma_bytes(bi):
    g = np.random.default_rng(42)
    a = rand_limbs(g, 16, 4096)
    b = rand_limbs(g, 16, 4096)
    p1 = host(_mul(bi, dev(a), dev(b), "plain"))
    for algo in ("mfma7", "mfma8"):
        assert np.array_equal(p1, host(_mul(bi, dev(a), dev(b), algo))), algo


def test_repeat_deterministic(bi):
    g = np.random.default_rng(43)
    a = dev(rand_limbs(g, 8, 5000))
    b = dev(rand_limbs(g, 8, 5000))
    for algo in ("mfma7", "mfma8"):
        r1 = host(_mul(bi, a, b, algo))
        r2 = host(_mul(bi, a, b, algo))
        assert np.array_equal(r1, r2)


def test_autotune_table_roundtrip(bi, orc, tmp_path):
    import json
    path = str(tmp_path / "tune.json")
    bi.autotune(path)
    t = json.load(open(path))
    assert t["op"] == "mul_mfma" and len(t["bins"]) == 8
    for e in t["bins"]:
        assert e["strips_per_band"] in (4, 8, 16, 32) and e["waves"] in (1, 4, 8)
        assert e["digit_bits"] in (7, 8) and e["tile"] in (16, 32)
        if e["waves"] == 1:
            assert e["digit_bits"] == 8 and e["strips_per_band"] in (4, 8) and e["tile"] == 16
        if e["tile"] == 32:
            assert e["digit_bits"] == 8 and e["strips_per_band"] in (8, 16, 32)
        else:
            assert e["strips_per_band"] != 32
    bi.autotune_load(path)
    try:
        g = np.random.default_rng(9)
        for n in (5000, 300):
            a = rand_limbs(g, 3, n)
            b = rand_limbs(g, 3, n)
            p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
            for i in range(3):
                assert np.array_equal(p[i], orc.mul1(a[i], b[i]))
    finally:
        bi.autotune_load(None)          # the built-in table again
    assert bi.mfma_config(16384, 16384) == (16, 8, 8)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,m", [(16384, 1), (16384, 3), (4096, 2), (1000, 7), (57, 1), (113, 2)])
def test_products_with_long_all_ones_runs(bi, orc, algo, n, m):
    # (B^n - 1) * b = b B^n - b: the low n limbs are B^n - b, all ones above
    # the lowest limbs, so carries between strips run through whole strips
    g = np.random.default_rng(n + m)
    a = np.full((2, n), 0xFFFFFFFF, np.uint32)
    b = rand_limbs(g, 2, m)
    b[1, 0] = 1
    b[1, 1:] = 0
    p = host(_mul(bi, dev(a), dev(b), algo))
    for i in range(2):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i])), i


def test_closing_scan_limbs_from_lds_or_global(bi, orc):
    """The closing strip carry scan takes every strip's limbs 0-1 from LDS in
    the uniform kernel where they fit (2^19 bits) and from global memory in a
    ragged plan's split segment: the same bytes, with carries that run through
    whole strips (all-ones operands, (B^n - 1) * small) included."""
    import torch
    n = 16384
    g = np.random.default_rng(1921)
    a = rand_limbs(g, 4, n)
    b = rand_limbs(g, 4, n)
    a[0] = 0xFFFFFFFF
    b[0] = 0xFFFFFFFF
    a[1] = 0xFFFFFFFF
    b[1, 1:] = 0
    b[1, 0] = 7
    a[2, : n // 2] = 0xFFFFFFFF
    bi.set_mfma_config(0, 0, 8)   # a forced configuration: the uniform kernel, not split
    try:
        uni = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
    finally:
        bi.set_mfma_config(0, 0, 0)
    lens = np.full(4, n, np.int64)
    off = np.arange(5, dtype=np.int64) * n
    plan = bi.MulPlan(lens, lens)
    assert plan.segments()[0]["parts"] > 1
    out, oo = plan(dev(a.reshape(-1)), torch.from_numpy(off).cuda(), dev(b.reshape(-1)),
                   torch.from_numpy(off).cuda())
    rag = host(out).reshape(4, 2 * n)
    plan.close()
    assert np.array_equal(uni, rag)
    want = oracle_map(lambda i: orc.mul1(a[i], b[i]), range(4))
    assert all(np.array_equal(uni[i], want[i]) for i in range(4))


@pytest.mark.parametrize("dw,n", [(7, 16397), (8, 18432), (0, 18432)])
def test_largest_supported_size(bi, orc, dw, n):
    # 16,397 limbs: the largest 7-bit-digit operands whose digits fit the LDS
    # with 8 waves; 18,432 = BIGINT_MFMA_MAX_LIMBS (8-bit digits, also the
    # default there)
    g = np.random.default_rng(dw)
    a = rand_limbs(g, 1, n)
    b = rand_limbs(g, 1, n)
    bi.set_mfma_config(0, 8, dw)
    try:
        p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))[0]
    finally:
        bi.set_mfma_config(0, 0, 0)
    assert np.array_equal(p, orc.mul1(a[0], b[0]))


def test_forced_7bit_beyond_lds_is_unsupported(bi):
    a = dev(np.zeros((1, 16398), np.uint32))
    bi.set_mfma_config(0, 8, 7)
    try:
        with pytest.raises(bi.BigIntError) as e:
            bi.mul(a, a, bi.MUL_MFMA)
        assert e.value.code == bi.EUNSUPPORTED
    finally:
        bi.set_mfma_config(0, 0, 0)


@pytest.mark.parametrize("pat", ["zeros", "zeros_ones", "alt"])
def test_offset_digit_extremes(bi, orc, pat):
    # offset 8-bit digits: zero bytes are -128, 0xFF bytes +127, so zero
    # operands drive every MFMA sum to its largest magnitude (2^14 per pair at
    # the deepest column of the largest size)
    n = 18432
    a = np.zeros((1, n), np.uint32)
    b = np.zeros((1, n), np.uint32)
    if pat == "zeros_ones":
        b[:] = 0xFFFFFFFF
    elif pat == "alt":
        a[:] = 0x00FF00FF
        b[:] = 0xFF00FF00
    p = host(_mul(bi, dev(a), dev(b), "mfma8"))[0]
    assert np.array_equal(p, orc.mul1(a[0], b[0]))


# ---- one Karatsuba level over the MFMA-split multiply ----------------------------------

@pytest.mark.parametrize("n", [2, 3, 8, 12, 64, 65, 127, 1000, 1001, 1004, 4096, 8200, 16384, 18432])
def test_karatsuba(bi, orc, n):
    g = np.random.default_rng(n + 77)
    a = rand_limbs(g, 6, n)
    b = rand_limbs(g, 6, n)
    h = (n + 1) // 2
    a[1] = 0xFFFFFFFF
    b[1] = 0xFFFFFFFF                      # largest operands
    a[2, h:] = a[2, :n - h]                # a1 = low part of a0: a0 - a1 mostly 0 limbs
    if 2 * h == n:
        a[3, h:] = a[3, :h]                # a0 == a1: the middle sign is 0
    b[4, :h] = 0                           # b0 = 0: b1 - b0 = b1 > 0
    a[5, :h] = 0                           # a0 = 0 < a1: negative difference
    b[5, h:] = 0                           # b1 = 0 < b0: negative difference, sign +1
    p = host(bi.mul(dev(a), dev(b), bi.MUL_KARATSUBA))
    for i in range(6):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i])), i


def test_karatsuba_matches_mfma_bytes(bi):
    from paper_2607_28897_amd import inputs
    c = inputs.pairs_2e19()
    ta, tb = dev(c["a"]), dev(c["b"])
    assert np.array_equal(host(bi.mul(ta, tb, bi.MUL_KARATSUBA)), host(bi.mul(ta, tb, bi.MUL_MFMA)))


def test_karatsuba_unsupported_shapes(bi):
    g = np.random.default_rng(1)
    with pytest.raises(bi.BigIntError):
        bi.mul(dev(rand_limbs(g, 1, 10)), dev(rand_limbs(g, 1, 11)), bi.MUL_KARATSUBA)
    with pytest.raises(bi.BigIntError):
        bi.mul(dev(rand_limbs(g, 1, 1)), dev(rand_limbs(g, 1, 1)), bi.MUL_KARATSUBA)


@pytest.mark.parametrize("P", [4, 8])
@pytest.mark.parametrize("na,nb,B", [(1, 1, 7), (2, 3, 5), (17, 5, 9), (64, 64, 13), (128, 128, 33),
                                     (256, 200, 10), (512, 512, 9), (700, 1, 3), (2048, 2048, 2),
                                     (3000, 1096, 2)])
def test_one_wave_per_instance(bi, orc, P, na, nb, B):
    """Several instances per work-group, one wave each (waves = 1), including
    a batch that does not fill the last work-group, unequal operands, the
    size limit (na + nb = 4096 limbs), all-ones rows and the low product."""
    g = np.random.default_rng(na * 7 + nb + P)
    a = rand_limbs(g, B, na)
    b = rand_limbs(g, B, nb)
    a[0] = 0xFFFFFFFF
    b[0] = 0xFFFFFFFF
    if B > 1:
        a[1] = 0
    bi.set_mfma_config(P, 1, 8)
    try:
        assert bi.mfma_config(na, nb) == (P, 1, 8)
        p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
        lo = host(bi.mullo(dev(a), dev(a))) if na <= 2048 else None
    finally:
        bi.set_mfma_config(0, 0, 0)
    for i in range(B):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i])), i
        if lo is not None:
            assert np.array_equal(lo[i], orc.mul1(a[i], a[i])[:na]), i


@pytest.mark.parametrize("n", [128, 256])
def test_batch_decides_waves(bi, orc, n):
    """Uniform batches from n*n/64 instances up (products mod B^n: n*n/256,
    Poly: n*n/16) run the table's one-wave-per-instance kernel, smaller ones
    4 waves per instance: the rows of a batch at the threshold and of one just
    below it must be the same bytes, and sampled rows the oracle's."""
    g = np.random.default_rng(n + 11)
    assert bi.mfma_config(n, n)[1] == 1
    for B, ops in ((n * n // 64, ("mul",)), (n * n // 256, ("mullo",)), (n * n // 16, ("poly",))):
        a = rand_limbs(g, B, n)
        b = rand_limbs(g, B, n)
        a[0] = 0xFFFFFFFF
        b[0] = 0xFFFFFFFF
        ta, tb = dev(a), dev(b)
        for op in ops:
            f = {"mul": lambda x, y: bi.mul(x, y, bi.MUL_MFMA), "mullo": bi.mullo, "poly": bi.poly}[op]
            ref = {"mul": orc.mul1, "mullo": orc.mullo1, "poly": orc.poly1}[op]
            big = host(f(ta, tb))
            small = host(f(ta[:B - 1], tb[:B - 1]))
            assert np.array_equal(big[:B - 1], small), op
            for i in (0, 1, B // 2, B - 2, B - 1):
                assert np.array_equal(big[i], ref(a[i], b[i])), (op, i)


@pytest.mark.parametrize("na,nb", [(1024, 1024), (700, 1500), (1500, 700), (33, 2000), (2048, 2048)])
def test_plain_split_parts_match_whole_blocks(bi, orc, na, nb):
    """Small batches run the plain product with every block's common range
    cut into parts summed by different waves; the same pairs inside a batch
    large enough to fill the chip run whole blocks.  Both equal the oracle."""
    g = np.random.default_rng(na * 3 + nb)
    a = rand_limbs(g, 4, na)
    b = rand_limbs(g, 4, nb)
    a[1] = 0xFFFFFFFF                      # every column at its largest
    b[1] = 0xFFFFFFFF
    b[2] = 0
    small = host(bi.mul(dev(a), dev(b), bi.MUL_PLAIN))
    big_a = np.concatenate([a, rand_limbs(g, 2044, na)])
    big_b = np.concatenate([b, rand_limbs(g, 2044, nb)])
    big = host(bi.mul(dev(big_a), dev(big_b), bi.MUL_PLAIN))[:4]
    assert np.array_equal(small, big)
    for i in range(4):
        assert np.array_equal(small[i], orc.mul1(a[i], b[i])), i


def test_unaligned_buffers_take_the_scalar_paths(bi, orc):
    """Operands and outputs 4 bytes past a 16-byte boundary: add, sub and the
    Karatsuba passes fall back from 16-byte accesses to limb-by-limb ones and
    give the same bytes."""
    import ctypes
    import torch
    L = bi.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = np.random.default_rng(4242)
    n, B = 1024, 3
    a = rand_limbs(g, B, n)
    b = rand_limbs(g, B, n)
    a[1] = 0xFFFFFFFF
    b[1] = 0xFFFFFFFF
    ta = torch.zeros(B * n + 1, dtype=torch.int32, device="cuda")
    tb = torch.zeros(B * n + 1, dtype=torch.int32, device="cuda")
    ta[1:] = torch.from_numpy(a.reshape(-1).view(np.int32)).cuda()
    tb[1:] = torch.from_numpy(b.reshape(-1).view(np.int32)).cuda()
    out = torch.zeros(B * 2 * n + 1, dtype=torch.int32, device="cuda")
    cy = torch.zeros(B, dtype=torch.int32, device="cuda")
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + 4 * off)
    assert L.bigint_mul(P(out, 1), P(ta, 1), n, P(tb, 1), n, B, bi.MUL_KARATSUBA, s) == 0
    got = out[1:].cpu().numpy().view(np.uint32).reshape(B, 2 * n)
    for i in range(B):
        assert np.array_equal(got[i], orc.mul1(a[i], b[i])), i
    assert L.bigint_add(P(out, 1), P(cy), P(ta, 1), P(tb, 1), n, B, s) == 0
    got = out[1:1 + B * n].cpu().numpy().view(np.uint32).reshape(B, n)
    want, wc = orc.add(a, b)
    assert np.array_equal(got, want) and np.array_equal(cy.cpu().numpy().view(np.uint32), wc)
    assert L.bigint_sub(P(out, 1), P(cy), P(ta, 1), P(tb, 1), n, B, s) == 0
    got = out[1:1 + B * n].cpu().numpy().view(np.uint32).reshape(B, n)
    want, wc = orc.sub(a, b)
    assert np.array_equal(got, want) and np.array_equal(cy.cpu().numpy().view(np.uint32), wc)


@pytest.mark.parametrize("P,waves", [(8, 4), (8, 8), (16, 4), (16, 8)])
@pytest.mark.parametrize("na,nb", [(1, 1), (3, 700), (64, 64), (257, 255), (1000, 1000), (4097, 4095),
                                   (12000, 300), (16384, 16384), (18432, 18432)])
def test_tile32_shapes(bi, orc, P, waves, na, nb):
    """32x32x32 tiles (four strips per tile, 32 phases per band) on every
    strips-per-band and wave count they take: ragged tails, unequal
    operands and the largest size, against the oracle."""
    g = np.random.default_rng(na * 31 + nb + P + waves)
    B = 2 if na * nb > 10**7 else 3
    a = rand_limbs(g, B, na)
    b = rand_limbs(g, B, nb)
    b[B - 1] = 0xFFFFFFFF
    bi.set_mfma_config(P, waves, 8)
    bi.set_mfma_tile(32)
    try:
        p = host(bi.mul(dev(a), dev(b), bi.MUL_MFMA))
    finally:
        bi.set_mfma_config(0, 0, 0)
        bi.set_mfma_tile(0)
    for i in range(B):
        assert np.array_equal(p[i], orc.mul1(a[i], b[i])), i


@pytest.mark.parametrize("pat", [0x00000000, 0xFFFFFFFF, 0x80808080, 0x7F7F7F7F])
def test_tile32_offset_digit_extremes(bi, orc, pat):
    """Every offset digit at -128, +127, 0 or -1: the largest MFMA sums."""
    n = 16384
    a = np.full((1, n), pat, np.uint32)
    bi.set_mfma_tile(32)
    try:
        p = host(bi.mul(dev(a), dev(a), bi.MUL_MFMA))[0]
    finally:
        bi.set_mfma_tile(0)
    assert np.array_equal(p, orc.mul1(a[0], a[0]))


@pytest.mark.parametrize("n", [700, 4096, 16384])
def test_tile32_mullo(bi, orc, n):
    """Products mod B^n (only the strips below limb n) on 32x32 tiles."""
    g = np.random.default_rng(n + 5)
    a = rand_limbs(g, 2, n)
    b = rand_limbs(g, 2, n)
    bi.set_mfma_tile(32)
    try:
        p = host(bi.mullo(dev(a), dev(b)))
    finally:
        bi.set_mfma_tile(0)
    for i in range(2):
        assert np.array_equal(p[i], orc.mullo1(a[i], b[i])), i


def test_tile_query_and_errors(bi):
    assert bi.lib().bigint_set_mfma_tile(24) == bi.EINVAL
    bi.set_mfma_tile(32)
    try:
        bi.set_mfma_config(16, 8, 8)
        assert bi.mfma_tile(16384, 16384) == 32
        bi.set_mfma_config(4, 8, 8)            # 4 strips per band: not a whole tile
        assert bi.mfma_tile(16384, 16384) == 16
        bi.set_mfma_config(16, 8, 7)           # 7-bit digits run 16x16 tiles
        assert bi.mfma_tile(16384, 16384) == 16
    finally:
        bi.set_mfma_config(0, 0, 0)
        bi.set_mfma_tile(0)

