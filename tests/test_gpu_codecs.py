"""The device codecs of the 16-bit storage formats: bfloat16 rounding by the gfx950 conversion
instruction equals integer rounding to nearest even on every one of the 2^32 float32 patterns (the
host codec, which the CPU tests pin to the definition, computes the same integer rounding); binary16
equals NumPy's float16 on a sample with every halfway case; decoding is exact on all 65536 patterns."""
import numpy as np
import pytest
import torch

from parity_util import announce
from test_codecs import _sample

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def test_bf16_all_float32_patterns(mrh):
    announce("bf16 device conversion on all 2^32 float32 patterns")
    n = 1 << 28
    for start in range(0, 1 << 32, n):
        u = torch.arange(start, start + n, dtype=torch.int64, device="cuda")
        x = torch.where(u >= (1 << 31), u - (1 << 32), u).to(torch.int32).view(torch.float32)
        got = mrh.convert(x, "bf16").to(torch.int64) & 0xFFFF
        nan = (u & 0x7FFFFFFF) > 0x7F800000
        ref = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
        bad = (~nan & (got != ref)) | (nan & ((got & 0x7FFF) <= 0x7F80))
        assert int(bad.sum()) == 0, (start, int(bad.sum()))
        del u, x, got, nan, ref, bad


def test_f16_encode_and_decode(mrh):
    announce("f16 / bf16 device conversions against NumPy and the host codec")
    x = _sample(seed=2)
    got = mrh.convert(torch.from_numpy(x).cuda(), "f16").cpu().numpy().view(np.uint16)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    nan = np.isnan(x)
    assert np.all(np.isnan(got[nan].view(np.float16)))
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.array_equal(got[~nan], mrh.convert(x, "f16")[~nan])
    b = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    for st in ("f16", "bf16"):
        dev = mrh.convert(torch.from_numpy(b.view(np.int16)).cuda(), st, decode=True).cpu().numpy()
        host = mrh.convert(b, st, decode=True)
        same = (dev.view(np.uint32) == host.view(np.uint32)) | (np.isnan(dev) & np.isnan(host))
        assert same.all(), st
