"""Launch parameters and autotuning: every tuning point gives the oracle's
bytes; the tuner keeps the fastest point and writes the tune cache."""

import json
import os
import sys

import numpy as np
import pytest

from oracle import cref
import workloads as W

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


def test_every_tune_point_gives_the_oracle_bytes(bz):
    import torch
    b = W.config4(nb=60, lo=500, hi=300_000, seed=81)
    x = torch.from_numpy(b.data).cuda()
    want = cref.compress(b.data, b.offsets, 9, threads=16)
    ctx = bz.Context()
    try:
        for cs in (1, 24, 48, 96, 1024):
            for mc in (2048, 4096):
                for ag in (128, 512):
                    _say(f"tune point mtf_chunk={mc} assign_groups={ag} count_steps={cs}")
                    ctx.set_tune(mc, ag, cs)
                    z = bz.Compressor(ctx=ctx)(x, b.offsets, level=9).cpu().numpy().tobytes()
                    assert z == want, (mc, ag, cs)
        ctx.set_tune()
    finally:
        ctx.close()


def test_tuner_writes_cache_and_new_context_reads_it(bz, tmp_path):
    import torch
    b = W.config2(total=3_000_000, block=300_000, seed=82)
    x = torch.from_numpy(b.data).cuda()
    path = str(tmp_path / "tune.json")
    ctx = bz.Context(tune_cache=path)
    _say("bzg_tune on a 3 MB batch")
    chosen = ctx.tune(x, b.offsets, 9)
    assert chosen[0] in (2048, 4096) and chosen[1] in (128, 512) and chosen[2] in (24, 48, 96)
    ctx.close()
    entries = json.load(open(path))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("gfx") and (val["mtf_chunk"], val["assign_groups"], val["count_steps"]) == chosen
    ctx2 = bz.Context(tune_cache=path)
    z = bz.Compressor(ctx=ctx2)(x, b.offsets, level=9).cpu().numpy().tobytes()
    assert z == cref.compress(b.data, b.offsets, 9, threads=16)
    ctx2.close()


def test_bad_tune_values(bz):
    ctx = bz.Context()
    for args in ((1000, 0, 0), (0, 256, 0), (0, 0, 5000)):
        with pytest.raises(bz.BzgError) as ei:
            ctx.set_tune(*args)
        assert ei.value.code == bz.native.BZG_EINVAL
    ctx.close()
