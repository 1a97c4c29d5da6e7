"""GPU parity of programs over relations of arity up to 4 (the paper's
requirement R3, multiple join columns, Section 3; joins on several columns,
Section 5.1), bit-exact against the oracle: the paper's Foo/Bar example, a
recursive rule whose join key has two columns, a 4-column head built by a
chain of joins, and random programs over relations of arity 1-4 (the
generator the oracle's brute-force pins use), with 32- and 64-bit keys, hash
and learned probes."""

import os
import random
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))
from test_oracle_wide import (ARITY, IDBS, as_arrays, random_wide_edb,  # noqa: E402
                              random_wide_program, render)


def say(msg):
    print(msg, flush=True)


def gpu_eval(program, edb, idb, **kw):
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    return pkg.evaluate(program, edb, idb, device=0, stream=torch.cuda.current_stream(), **kw)


def check_same(program, edb, idb, **kw):
    want = oracle.evaluate(program, edb, idb, max_iterations=100_000)
    rels, deltas, st = gpu_eval(program, edb, idb, **kw)
    for name in idb:
        assert np.array_equal(rels[name], want.relations[name]), (name, program)
        assert deltas[name] == want.deltas[name], (name, program)
    return rels, st


def fixture(name):
    out = {}
    for ln in open(os.path.join(ROOT, "tests", "golden", name)):
        ln = ln.strip()
        if ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            out.setdefault(k.strip(), []).append(v.strip())
    return out


@pytest.mark.parametrize("learned", [False, True])
def test_foobar_paper_example(learned):
    say(f"foobar, learned={learned}")
    fx = fixture("foobar_paper_example.txt")
    rows = lambda s: np.array([[int(x) for x in t.split()] for t in s.split(",")], np.uint32)
    edb = {"Foo": rows(fx["foo"][0]), "Bar": rows(fx["bar"][0])}
    rels, st = check_same("Foobar(c, d) :- Foo(a, b, c), Bar(a, b, d).", edb, {"Foobar": 2},
                          learned=learned)
    assert {tuple(r) for r in rels["Foobar"].tolist()} == {(5, 1), (2, 1)}


@pytest.mark.parametrize("spread", [False, True])
@pytest.mark.parametrize("learned", [False, True])
def test_same_label_reachability(spread, learned):
    """P(x, z, l) :- P(x, y, l), E(y, z, l): a recursive rule whose join key
    is the pair (y, l).  With spread ids (up to 2^20) the tuples take 60 of
    64 key bits."""
    say(f"same-label reach, spread={spread}, learned={learned}")
    rng = np.random.default_rng(7)
    n, labels, m = 3000, 4, 9000
    E = np.stack([rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, labels, m)], 1)
    if spread:
        E = E * 331 + 17
    E = E.astype(np.uint32)
    prog = "P(x, y, l) :- E(x, y, l).\nP(x, z, l) :- P(x, y, l), E(y, z, l)."
    rels, st = check_same(prog, {"E": E}, {"P": 3}, learned=learned)
    assert st.key_bytes == 8 and len(rels["P"]) > m


def test_four_column_head_and_filters():
    """A 4-column head from a chain of two joins, a unary EDB, a filter
    across the join and a variable repeated in one atom."""
    say("four columns")
    rng = np.random.default_rng(11)
    A = rng.integers(0, 60, (400, 2)).astype(np.uint32)
    B = rng.integers(0, 60, (400, 3)).astype(np.uint32)
    B[:50, 2] = B[:50, 1]
    U = np.unique(rng.integers(0, 60, (30, 1))).reshape(-1, 1).astype(np.uint32)
    prog = """W(a, b, c, d) :- A(a, b), B(b, c, d), a != d.
W(a, b, c, c) :- B(a, b, c), U(a).
V(x, y) :- B(x, y, y).
T(x) :- W(x, y, z, t), U(t)."""
    check_same(prog, {"A": A, "B": B, "U": U}, {"W": 4, "V": 2, "T": 1})


@pytest.mark.parametrize("learned", [False, True])
def test_cross_products_and_binary_fallback(learned):
    """Binary programs outside the chain-join form run as wide plans: cross
    products (a join with no shared column, whose inner is taken whole, also
    with the delta as outer), three variables live between joins, and joins
    whose carried tuple only has to exist."""
    say(f"cross products, learned={learned}")
    rng = np.random.default_rng(23)
    E = np.unique(rng.integers(0, 40, (120, 2)), axis=0).astype(np.uint32)
    F = np.unique(rng.integers(0, 40, (60, 2)), axis=0).astype(np.uint32)
    U = np.unique(rng.integers(0, 40, (6, 1)), axis=0).astype(np.uint32)
    prog = """X(x, y) :- E(x, a), F(y, b), a != b.
B(x, y) :- U(x), U(y).
T(x, y) :- E(x, a), E(a, b), E(b, y), E(x, y), E(a, y), E(b, x).
C(x, y) :- E(x, y), F(a, b), U(a).
P(x, y) :- U(x), U(y).
P(x, z) :- P(x, y), F(y, z).
P(x, z) :- P(x, y), U(z), x != z."""
    check_same(prog, {"E": E, "F": F, "U": U},
               {"X": 2, "B": 2, "T": 2, "C": 2, "P": 2}, learned=learned)


@pytest.mark.parametrize("spread", [False, True])
def test_random_wide_programs(spread):
    """Random programs over relations of arity 1-4 against the oracle; the
    planner rejects only bodies that keep more than four variables live
    between joins."""
    import paper_2311_02206_amd as pkg
    rng = random.Random(99 + spread)
    ran = 0
    for k in range(120):
        rules = random_wide_program(rng)
        edb = random_wide_edb(rng, n_ids=rng.randint(3, 9))
        arr = as_arrays(edb)
        if spread:  # ids up to about 2^15: four columns fill 60 key bits
            arr = {r: (a.astype(np.uint64) * 2711 + 5).astype(np.uint32) for r, a in arr.items()}
        try:
            check_same(render(rules), arr, {r: ARITY[r] for r in IDBS},
                       learned=bool(k % 2))
            ran += 1
        except pkg.HlError as e:
            assert e.code == pkg.hisalog.HL_E_UNSUPPORTED, (render(rules), e)
    say(f"random wide programs run: {ran}")
    assert ran >= 110


def test_wide_limits():
    """Tuples that would need keys wider than 64 bits are refused."""
    import paper_2311_02206_amd as pkg
    E = np.array([[1, 2, 1 << 30]], np.uint32)
    with pytest.raises(pkg.HlError) as ei:
        gpu_eval("P(x, y, z) :- E(x, y, z).", {"E": E}, {"P": 3})
    assert ei.value.code == pkg.hisalog.HL_E_UNSUPPORTED
