"""Field codecs on the GPU (Sec. 2.1 null suppression and Elias delta,
Sec. 3.5 GFC-style float delta): streams byte for byte against the oracle,
and decoding back to the values."""

import math
import random
import struct
import sys

import numpy as np
import pytest

from oracle import fields as F

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bz():
    import torch
    import paper_1109_2348_amd as bz
    assert torch.cuda.is_available()
    return bz


def _ints(n, seed):
    rnd = random.Random(seed)
    # a field mix: small counters, ids, occasional large values and zeros
    out = []
    for i in range(n):
        r = rnd.random()
        out.append(0 if r < 0.1 else rnd.getrandbits(7) if r < 0.5 else rnd.getrandbits(15) if r < 0.8
                   else rnd.getrandbits(24) if r < 0.95 else rnd.getrandbits(32))
    return out


def _doubles(n, seed):
    rnd = random.Random(seed)
    x, out = 0.0, []
    for i in range(n):
        # a smooth signal with noise, and a few special values
        x += rnd.gauss(0, 0.01)
        v = math.sin(i / 50.0) * 100.0 + x
        r = rnd.random()
        out.append(v if r > 0.01 else rnd.choice([0.0, -0.0, math.inf, -math.inf, float("nan"), 5e-324]))
    return out


SIZES = [1, 1000, 4095, 4096, 4097, 70001]


@pytest.mark.parametrize("n", SIZES)
def test_integer_codecs_equal_oracle(bz, n):
    import torch
    from paper_1109_2348_amd import native
    vals = _ints(n, seed=n)
    t = torch.tensor(np.array(vals, dtype=np.uint32).view(np.int32)).cuda()
    for codec, enc in ((native.FIELD_NS32, F.ns_encode), (native.FIELD_EDELTA32, F.edelta_encode)):
        _say(f"codec {codec}, {n} values")
        z = bz.field_encode(t, codec)
        want = enc(vals)
        assert z.cpu().numpy().tobytes() == want
        back = bz.field_decode(z, codec, n)
        assert np.array_equal(back.cpu().numpy().view(np.uint32), np.array(vals, np.uint32))


@pytest.mark.parametrize("n", SIZES)
def test_gfc_equals_oracle(bz, n):
    import torch
    from paper_1109_2348_amd import native
    vals = _doubles(n, seed=n)
    t = torch.tensor(vals, dtype=torch.float64).cuda()
    _say(f"gfc, {n} values")
    z = bz.field_encode(t, native.FIELD_GFC64)
    assert z.cpu().numpy().tobytes() == F.gfc_encode(vals)
    back = bz.field_decode(z, native.FIELD_GFC64, n)
    want = np.array([struct.unpack("<Q", struct.pack("<d", v))[0] for v in vals], np.uint64)
    assert np.array_equal(back.cpu().numpy().view(np.uint64), want)


def test_extremes_and_errors(bz):
    import torch
    from paper_1109_2348_amd import native
    vals = [0, (1 << 32) - 1] * 3000
    t = torch.tensor(np.array(vals, dtype=np.uint32).view(np.int32)).cuda()
    for codec, enc in ((native.FIELD_NS32, F.ns_encode), (native.FIELD_EDELTA32, F.edelta_encode)):
        z = bz.field_encode(t, codec)
        assert z.cpu().numpy().tobytes() == enc(vals)
        assert np.array_equal(bz.field_decode(z, codec, len(vals)).cpu().numpy().view(np.uint32),
                              np.array(vals, np.uint32))
    # a stream cut short: reported, not read past its end
    z = bz.field_encode(t, native.FIELD_NS32)
    _say("decode a truncated NS32 stream")
    with pytest.raises(bz.BzgError) as ei:
        bz.field_decode(z[:-100], native.FIELD_NS32, len(vals))
    assert ei.value.code == native.BZG_EDATA
