"""The 16-bit storage conversions on the host (no GPU): binary16 against NumPy's float16, bfloat16
against rounding to nearest, ties to even, written from its definition (the nearer of the two
bfloat16 neighbours in exact float64 arithmetic, the one with an even last bit on a tie).  Decoding
is exact for every one of the 65536 patterns."""
import numpy as np
import pytest

import paper_2511_21459_amd as mrh

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


def _floats(b):
    return np.asarray(b, np.uint32).view(np.float32)


def bf16_from_definition(x):
    """Nearest bfloat16 (ties to even) of float32 x as a bit pattern; NaN -> any NaN (not checked)."""
    u = _bits(x).astype(np.uint64)
    sign = (u >> 31) << 15
    mag = u & 0x7FFFFFFF
    lo = mag >> 16                          # truncated magnitude, a bfloat16 pattern
    hi = lo + 1                             # the next larger bfloat16 magnitude (0x7F80 is infinity)
    val = lambda p: _floats((p << 16).astype(np.uint32)).astype(np.float64)
    a = _floats(mag.astype(np.uint32)).astype(np.float64)
    with np.errstate(invalid="ignore"):
        dlo = a - val(lo)
        dhi = np.where(hi >= 0x7F80, np.inf, val(np.minimum(hi, 0x7F7F)) - a)
        # past the largest finite value the upper neighbour is infinity, reached from the halfway
        # point 0x7F7F8000 on (round to nearest, ties to even, with the exponent range unbounded)
        over = (hi == 0x7F80) & (mag >= 0x7F7F8000)
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    pick = np.where(over, 0x7F80, pick)
    pick = np.where(mag >= 0x7F800000, lo, pick)  # infinity stays infinity (NaN handled apart)
    return (sign | pick).astype(np.uint16)


def _sample(n=1 << 20, seed=0):
    rng = np.random.default_rng(seed)
    raw = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    # exact halfway points and their neighbours for both formats, subnormals, extremes
    k = rng.integers(0, 1 << 16, size=4096, dtype=np.uint64).astype(np.uint32)
    half_bf = (k << 16) | 0x8000
    f16 = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16).astype(np.float32)
    f16 = f16[np.isfinite(f16)]
    nxt = np.nextafter(f16, np.float32(np.inf))
    mids = ((f16.astype(np.float64) + np.nextafter(f16.astype(np.float16), np.float16(np.inf)).astype(np.float64)) / 2)
    mids = mids[np.isfinite(mids)].astype(np.float32)
    special = np.array([0.0, -0.0, 65504.0, 65519.996, 65520.0, -65520.0, 6.1e-5, 5.96e-8, 2.98e-8, 1e-45, 3.4028235e38,
                        np.inf, -np.inf, np.nan], np.float32)
    return np.concatenate([_floats(raw), _floats(half_bf), _floats(half_bf - 1), _floats(half_bf + 1), mids,
                           np.nextafter(mids, np.float32(np.inf)), np.nextafter(mids, np.float32(-np.inf)), nxt, special])


def test_decode_all_patterns():
    b = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    f = mrh.convert(b, "f16", decode=True)
    ref = b.view(np.float16).astype(np.float32)
    assert np.array_equal(np.isnan(f), np.isnan(ref))
    assert np.array_equal(f[~np.isnan(ref)].view(np.uint32), ref[~np.isnan(ref)].view(np.uint32))
    g = mrh.convert(b, "bf16", decode=True)
    assert np.array_equal(g.view(np.uint32), b.astype(np.uint32) << 16)


def test_f16_encode_matches_numpy():
    x = _sample()
    got = mrh.convert(x, "f16")
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    nan = np.isnan(x)
    assert np.all(np.isnan(got[nan].view(np.float16)))
    assert np.array_equal(got[~nan], ref[~nan])


def test_bf16_encode_matches_definition():
    x = _sample(seed=1)
    got = mrh.convert(x, "bf16")
    ref = bf16_from_definition(x)
    nan = np.isnan(x)
    assert np.all((got[nan] & 0x7FFF) > 0x7F80)  # NaN stays NaN
    assert np.array_equal(got[~nan], ref[~nan])


def test_bf16_definition_pins():
    """The reference itself on hand-checked values: ties go to the even neighbour, the largest
    finite bfloat16 rounds up to infinity from its upper halfway point on, subnormals round like
    normals, the sign is kept."""
    cases = {0x3F808000: 0x3F80, 0x3F818000: 0x3F82, 0x3F808001: 0x3F81, 0x7F7F7FFF: 0x7F7F, 0x7F7F8000: 0x7F80,
             0x00008000: 0x0000, 0x00018000: 0x0002, 0x0000C000: 0x0001, 0xBF808001: 0xBF81, 0x7F800000: 0x7F80}
    x = _floats(np.array(list(cases), np.uint32))
    assert bf16_from_definition(x).tolist() == list(cases.values())


def test_codec_rejects_f32():
    with pytest.raises(ValueError):
        mrh.convert(np.zeros(3, np.float32), "f32")
