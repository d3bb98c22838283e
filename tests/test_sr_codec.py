"""The stochastically rounding FP16 encode of the RRMHD_STORE_F16_SR storage
codec.  The rule, written out here in numpy: with e the biased FP32 exponent
of x and m its 24-bit significand, d = max(126 - e, 13) bits are dropped, the
dropped fraction is kept to 13 bits (t = floor(m 2^(13-d))) and the kept
integer is k = floor((t + r_13) 2^-13) with r_13 the top 13 of the 32 random
bits; the FP16 pattern is the sign, then ((max(e, 113) - 113) << 10) + k
saturated at infinity; NaN stores a quiet NaN of its sign and the top ten
payload bits.
CPU: the rule is unbiased (the mean over all random bits is x itself),
reduces to round-down / round-up at the extreme random words, keeps FP16
values exactly and saturates past the range.  GPU: the library's encode equals the rule bit
for bit on 4 M values spanning every binade, FP16 subnormals, FP32
subnormals, overflow and special values."""
import numpy as np
import pytest


def sr_rule(x, r):
    x = np.ascontiguousarray(x, dtype=np.float32)
    r = np.ascontiguousarray(r, dtype=np.uint32).astype(np.uint64)
    b = x.view(np.uint32).astype(np.uint64)
    sign = (b >> np.uint64(16)) & np.uint64(0x8000)
    a = b & np.uint64(0x7FFFFFFF)
    e = (a >> np.uint64(23)).astype(np.int64)
    frac = a & np.uint64(0x7FFFFF)
    m = np.where(e > 0, frac | np.uint64(0x800000), frac)
    d = np.maximum(126 - e, 13)
    # the dropped fraction kept to 13 bits, plus the top 13 random bits
    t = np.where(d - 13 < 32, m >> np.minimum(d - 13, 31).astype(np.uint64), np.uint64(0))
    k = (t + (r >> np.uint64(19))) >> np.uint64(13)
    ex = (np.maximum(e, 113) - 113).astype(np.uint64) << np.uint64(10)
    h = np.minimum(ex + k, np.uint64(0x7C00))
    out = sign | h
    nan = a > np.uint64(0x7F800000)
    out[nan] = sign[nan] | np.uint64(0x7E00) | (frac[nan] >> np.uint64(13))
    return out.astype(np.uint16)


def f16_value(bits):
    return np.asarray(bits, dtype=np.uint16).view(np.float16).astype(np.float64)


def test_rule_is_unbiased_over_all_random_words():
    """The rule depends on the top 13 bits of r only.  Averaging the decoded
    result over those 8192 words gives x exactly in FP16's normal range; for
    FP16-subnormal results it gives x with its dropped fraction truncated to
    13 bits, within 2^-13 of the 2^-24 grid below x."""
    g = np.random.default_rng(1)
    words = (np.arange(1 << 13, dtype=np.uint64) << np.uint64(19)).astype(np.uint32)
    for lo, hi in ((-14, 15), (-18, -17), (-22, -21), (-30, -25)):
        xs = (g.uniform(1, 2, 40) * 2.0 ** g.integers(lo, hi, 40)).astype(np.float32)
        xs *= np.where(g.random(40) < 0.5, -1, 1).astype(np.float32)
        for x in xs:
            mean = f16_value(sr_rule(np.full(words.size, x), words)).mean()
            xd = float(x)
            if abs(xd) >= 2.0 ** -14:
                assert mean == xd, (x, mean)
            else:
                q = 2.0 ** -37  # 13 fraction bits of the subnormal grid 2^-24
                assert mean == np.sign(xd) * np.floor(abs(xd) / q) * q, (x, mean)
                assert abs(mean - xd) < q


def test_rule_extreme_words_and_exact_values():
    g = np.random.default_rng(2)
    x = (g.uniform(-1, 1, 10000) * 2.0 ** g.integers(-20, 15, 10000)).astype(np.float32)
    down = f16_value(sr_rule(x, np.zeros(x.size, np.uint32)))
    up = f16_value(sr_rule(x, np.full(x.size, 0xFFFFFFFF, np.uint32)))
    xd = x.astype(np.float64)
    # r = 0 truncates toward zero, r = 2^32 - 1 rounds away unless x is on the grid
    assert np.all(np.abs(down) <= np.abs(xd)) and np.all(np.abs(up) >= np.abs(xd))
    rn = x.astype(np.float16).astype(np.float64)
    assert np.all((down == rn) | (up == rn))
    # FP16 values are kept for every random word
    h = np.array([1.0, -2.5, 65504.0, 6.103515625e-05, 5.960464477539063e-08], np.float32)
    for w in (0, 1, 0x80000000, 0xFFFFFFFF):
        assert np.array_equal(f16_value(sr_rule(h, np.full(h.size, w, np.uint32))), h)
    # past the range: infinity; NaN: quiet NaN of its sign and payload; +-0 and tiny: zero
    assert np.all(sr_rule(np.array([7e4, -1e6, np.inf], np.float32),
                          np.array([0, 5, 0], np.uint32)) == np.array([0x7C00, 0xFC00, 0x7C00]))
    assert np.array_equal(sr_rule(np.array([np.nan, -np.nan], np.float32), np.zeros(2, np.uint32)),
                          np.array([0x7E00, 0xFE00], np.uint16))
    assert np.array_equal(sr_rule(np.array([0x7FFFFFFF, 0xFF800001], np.uint32).view(np.float32),
                                  np.zeros(2, np.uint32)), np.array([0x7FFF, 0xFE00], np.uint16))
    assert np.array_equal(sr_rule(np.array([0.0, -0.0, 1e-40], np.float32), np.full(3, 0xFFFFFFFF, np.uint32)),
                          np.array([0, 0x8000, 0], np.uint16))


def _inputs(n, seed):
    g = np.random.default_rng(seed)
    cat = np.arange(n) % 8
    e = np.where(cat < 5, g.integers(-40, 21, n),
                 np.where(cat == 5, g.integers(-27, -13, n), g.integers(14, 17, n)))
    bits = ((e + 127).astype(np.uint64) << np.uint64(23)) | g.integers(0, 1 << 23, n).astype(np.uint64)
    special = np.array([0x00000000, 0x3F800000, 0x477FE000, 0x38800000, 0x33800000,
                        0x7F800000, 0x7FC00000, 0x7F800001, 0x7FFFFFFF, 0x00000001, 0x007FFFFF,
                        0x00400000], dtype=np.uint64)
    bits = np.where(cat == 7, special[g.integers(0, special.size, n)], bits)
    bits ^= np.where(g.random(n) < 0.5, np.uint64(0x80000000), np.uint64(0))
    x = bits.astype(np.uint32).view(np.float32)
    r = g.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return x, r


@pytest.mark.gpu
def test_library_encode_equals_the_rule():
    torch = pytest.importorskip("torch")
    from paper_2602_14667_amd import rrmhd
    rrmhd.lib()
    print("[gpu] stochastic-rounding encode vs the rule", flush=True)
    x, r = _inputs(1 << 22, 3)
    got = rrmhd.sr_encode(torch.from_numpy(x).cuda(),
                          torch.from_numpy(r.view(np.int32)).cuda()).cpu().numpy().view(np.uint16)
    want = sr_rule(x, r)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(hex(int(x[i:i + 1].view(np.uint32)[0])), hex(int(r[i])),
                            hex(int(got[i])), hex(int(want[i]))) for i in bad[:8]]
