"""The LDS pad table of the contiguous multiply passes (vgf_lds_pads.hpp):
every entry keeps each line inside its pitch, is one-to-one, and keeps every
exchange access a per-lane base plus r times a constant (the form the
kernels address); and the committed table is the generator's output for a
sample of lengths (the full table takes about a minute to regenerate)."""
import os
import re
import types

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_08531_amd", "csrc")


def _gen():
    # loaded without writing a bytecode cache beside the library sources
    m = types.ModuleType("gen_lds_pads")
    path = os.path.join(CSRC, "gen_lds_pads.py")
    exec(compile(open(path).read(), path, "exec"), m.__dict__)
    return m


def _table():
    txt = open(os.path.join(CSRC, "vgf_lds_pads.hpp")).read()
    rows = re.findall(r"\{(-?\d+), (-?\d+), (-?\d+), (-?\d+), (-?\d+), (-?\d+)\},\s*// (\d+) / (\d+)", txt)
    return [tuple(int(x) for x in r) for r in rows]


def test_every_entry_fits_and_is_additive():
    g = _gen()
    table = _table()
    assert len(table) > 300
    for P, sign, e, nq, k, s, cost, base in table:
        f = lambda p: p + k * (p >> s)
        LP = P + P // 8
        assert len({f(p) for p in range(P)}) == P and f(P - 1) < LP, (P, sign, e, nq)
        assert cost <= base, (P, sign, e, nq)
        if (k, s) != (1, 3):
            c = g.evaluate(P, g.radices(P, sign), nq, e, k, s)
            assert c == cost, (P, sign, e, nq, c, cost)


@pytest.mark.parametrize("P", [64, 96, 256, 512])
def test_table_is_the_generator_output(P):
    g = _gen()
    table = {(r[0], r[1], r[2], r[3]): r[4:] for r in _table()}
    nq0 = g.wave_nq(P)
    for nq in sorted({nq0, max(1, nq0 // 2)}):
        for sign in (-1, 1):
            for e in range(len(g.radices(P, sign)) - 1):
                (c, k, s), base = g.best_pad(P, sign, e, nq)
                assert table[(P, sign, e, nq)] == (k, s, c, base), (P, sign, e, nq)
