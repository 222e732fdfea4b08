"""Pins of the oracle's precomputed-table mode (Sec. 4: tables computed
beforehand from data, no tree built per block), on the CPU."""

import bz2

import numpy as np
import pytest

from oracle import cref, ref
import workloads as W


def _data(total, block, seed):
    b = W.config2(total=total, block=block, seed=seed)
    return b.data, [int(o) for o in b.offsets]


def _fixed_example():
    """Two hand-made tables over the 258 symbols, both complete prefix codes:
    table 0 favours RUNA/RUNB (lengths 1, 2, then 9 for everything else up
    to a complete code), table 1 gives every symbol 8 or 9 bits.  Symbol 257
    (EOB of a full alphabet) gets a length no other entry of its table has
    near the end, so a wrong EOB mapping shows in the decoded tables."""
    t0 = [1, 2] + [0] * 256
    # remaining Kraft budget 1/4 over 256 symbols: 256 * 2^-10 = 1/4
    for v in range(2, 258):
        t0[v] = 10
    t1 = [8] * 258
    # 258 codes: 254 of length 8 and 4 of length 9 (254/256 + 4/512 = 1)
    for v in range(254, 258):
        t1[v] = 9
    return np.array([t0, t1], np.uint8)


def _kraft(lens):
    return sum(2.0 ** -int(x) for x in lens)


def test_example_tables_are_complete_codes():
    f = _fixed_example()
    assert _kraft(f[0]) == 1.0 and _kraft(f[1]) == 1.0


def test_fixed_streams_decode_with_stock_bz2_and_tiers_agree():
    data, offs = _data(9000, 3000, seed=11)
    f = _fixed_example()
    z1 = cref.compress(data, offs, 1, fixed=f)
    z0 = ref.compress(data.tobytes(), 1, offs, fixed=[list(map(int, t)) for t in f])
    assert z1 == z0
    assert bz2.decompress(z1) == data.tobytes()


def test_blocks_use_the_restriction_with_eob_from_symbol_257():
    data, offs = _data(6000, 2000, seed=12)
    f = _fixed_example()
    z = cref.compress(data, offs, 1, fixed=f)
    out, stages = ref.decompress(z, want_stages=True)
    assert out == data.tobytes()
    for st in stages:
        a = len(st["used"]) + 2
        assert len(st["lens"]) == 2
        for t in range(2):
            want = [int(f[t][v]) for v in range(a - 1)] + [int(f[t][257])]
            assert list(st["lens"][t]) == want


def test_selectors_are_cheapest_tables_lowest_on_ties():
    data, offs = _data(4000, 4000, seed=13)
    f = _fixed_example()
    same = np.array([f[1], f[1]], np.uint8)  # two equal tables: every group ties
    z = cref.compress(data, offs, 1, fixed=same)
    _, stages = ref.decompress(z, want_stages=True)
    assert all(s == 0 for st in stages for s in st["sel"])
    z = cref.compress(data, offs, 1, fixed=f)
    _, stages = ref.decompress(z, want_stages=True)
    for st in stages:
        syms = st["syms"]
        for j, s in enumerate(st["sel"]):
            grp = syms[j * 50:(j + 1) * 50]
            costs = [sum(st["lens"][t][x] for x in grp) for t in range(2)]
            assert costs[s] == min(costs) and (costs[0] > costs[1] or s == 0)


def test_tables_from_sample_tiers_agree():
    data, offs = _data(8000, 2000, seed=14)
    blocks = [data[offs[k]:offs[k + 1]] for k in range(len(offs) - 1)]
    c = cref.tables_from_sample(blocks)
    t = ref.tables_from_sample([ref.sample_symbols(blk.tobytes()) for blk in blocks])
    assert [list(map(int, r)) for r in c] == [list(r) for r in t]
    assert all(1 <= x <= 17 for r in t for x in r)
    assert all(abs(_kraft(r) - 1.0) < 1e-12 for r in t)


@pytest.mark.parametrize("seed", [21, 22])
def test_sample_tables_compress_other_data(seed):
    sample, so = _data(30000, 10000, seed=seed)
    fixed = cref.tables_from_sample([sample[so[k]:so[k + 1]] for k in range(len(so) - 1)])
    data, offs = _data(20000, 5000, seed=seed + 100)
    z = cref.compress(data, offs, 1, fixed=fixed)
    assert bz2.decompress(z) == data.tobytes()
