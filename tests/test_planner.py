"""CPU checks of the library's host logic on a planning-only engine
(device -1): parsing, the chain-join planner, and error codes."""

import os
import random
import sys

import pytest

import paper_2311_02206_amd as pkg
from paper_2311_02206_amd import hisalog as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))


def planner(decls):
    e = pkg.Engine(device=-1)
    for name, edb in decls:
        e.declare(name, 2, edb)
    return e


def code_of(fn):
    try:
        fn()
        return H.HL_OK
    except pkg.HlError as err:
        return err.code


@pytest.mark.parametrize("prog,decls", [
    ("reach", [("Edge", True), ("Reach", False)]),
    ("sg", [("Edge", True), ("SG", False)]),
    ("cspa_shaped", [("Assign", True), ("Dereference", True), ("ValueFlow", False),
                     ("ValueAlias", False), ("MemoryAlias", False)]),
])
def test_shipped_programs_plan(prog, decls):
    text = open(os.path.join(ROOT, "workloads", "programs", prog + ".dl")).read()
    with planner(decls) as e:
        e.program(text)


def test_error_codes():
    with planner([("E", True), ("R", False)]) as e:
        assert code_of(lambda: e.program("R(x, y) :- E(x, .")) == H.HL_E_INVALID
        assert code_of(lambda: e.program("R(x, y) :- Nope(x, y).")) == H.HL_E_INVALID
        assert code_of(lambda: e.program("R(x, _) :- E(x, y).")) == H.HL_E_INVALID
        assert code_of(lambda: e.program("R(x, w) :- E(x, y).")) == H.HL_E_INVALID
        assert code_of(lambda: e.program("E(x, y) :- R(x, y).")) == H.HL_E_INVALID
        assert code_of(lambda: e.program("R(x, y) :- E(x, y), a != y.")) == H.HL_E_INVALID
        # a cross product and three live variables are outside the binary
        # chain form: such programs are planned as wide ones
        assert code_of(lambda: e.program("R(x, y) :- E(x, a), E(y, b).")) == H.HL_OK
        assert code_of(lambda: e.program(
            "R(x, y) :- E(x, a), E(a, b), E(b, y), E(x, y), E(a, y), E(b, x).")) == H.HL_OK
        # five filters at one join are beyond both planners
        assert code_of(lambda: e.program(
            "R(x, y) :- E(x, a), E(a, y), x != y, x != a, a != y, y != x, a != x.")) == (
            H.HL_E_UNSUPPORTED)
        # shapes that reduce to equality tests are planned
        assert code_of(lambda: e.program("R(x, x) :- E(x, x).")) == H.HL_OK
        assert code_of(lambda: e.program("R(x, y) :- E(x, y), E(y, x).")) == H.HL_OK
        assert code_of(lambda: e.load("E", [[1, 2]])) == H.HL_E_STATE
        assert code_of(lambda: e.run()) == H.HL_E_STATE
        assert code_of(lambda: e.autotune()) == H.HL_E_STATE
    e = pkg.Engine(device=-1)
    assert code_of(lambda: e.declare("T", 5, False)) == H.HL_E_UNSUPPORTED
    assert code_of(lambda: e.declare("T", 0, False)) == H.HL_E_UNSUPPORTED
    assert code_of(lambda: e.declare("bad name", 2, False)) == H.HL_E_INVALID
    e.declare("T", 2, False)
    assert code_of(lambda: e.declare("T", 2, False)) == H.HL_E_INVALID
    e.close()


def test_random_programs_mostly_plan():
    from test_oracle_pins import random_program, render
    rng = random.Random(77)
    ok = unsupported = 0
    for _ in range(300):
        with planner([("E", True), ("F", True), ("P", False), ("Q", False)]) as e:
            c = code_of(lambda: e.program(render(random_program(rng))))
            assert c in (H.HL_OK, H.HL_E_UNSUPPORTED)
            ok += c == H.HL_OK
            unsupported += c == H.HL_E_UNSUPPORTED
    print("planned", ok, "unsupported", unsupported)
    assert ok == 300


def test_unary_relations_plan():
    """Unary relations: declared with arity 1, used in heads and bodies; a
    unary atom joins on its one column, never on its constant one."""
    e = pkg.Engine(device=-1)
    for name, ar, edb in (("E", 2, True), ("S", 1, True), ("R", 1, False), ("B", 2, False),
                          ("N", 1, False)):
        e.declare(name, ar, edb)
    e.program("R(x) :- S(x).\nR(y) :- R(x), E(x, y).\nN(x) :- E(x, _).\n"
              "B(x, y) :- R(x), E(y, x).\nN(x) :- E(x, x).\nB(x, x) :- R(x), S(x).\n")
    assert code_of(lambda: e.program("R(x, y) :- E(x, y).")) == H.HL_E_INVALID
    assert code_of(lambda: e.program("B(x) :- E(x, y).")) == H.HL_E_INVALID
    # two unary atoms with no shared variable: a cross product (wide plans)
    assert code_of(lambda: e.program("B(x, y) :- R(x), S(y).")) == H.HL_OK
    e.close()
    e = pkg.Engine(device=-1)
    assert code_of(lambda: e.declare("Z", 0, False)) == H.HL_E_UNSUPPORTED
    e.declare("U", 1, False)
    e.close()


def test_wide_programs_plan():
    """Relations of arity 3-4: joins on several columns, cross products and
    carried tuples of up to four variables are planned; five live variables
    are not."""
    e = pkg.Engine(device=-1)
    try:
        for name, ar, edb in (("Foo", 3, True), ("Bar", 3, True), ("E", 2, True),
                              ("Foobar", 2, False), ("P", 3, False), ("W", 4, False)):
            e.declare(name, ar, edb)
        e.program("Foobar(c, d) :- Foo(a, b, c), Bar(a, b, d).")
        e.program("P(x, y, l) :- Foo(x, y, l).\nP(x, z, l) :- P(x, y, l), Foo(y, z, l).")
        e.program("W(a, b, c, d) :- E(a, b), Foo(b, c, d), a != d.")
        assert code_of(lambda: e.program("P(a, b, c) :- E(a, b), E(c, d).")) == H.HL_OK
        assert code_of(lambda: e.program(
            "W(a, b, c, d) :- Foo(a, b, c), E(f, a), Foo(d, e, f), E(e, f).")) == (
            H.HL_E_UNSUPPORTED)
        assert code_of(lambda: e.program(
            "W(a, b, c, d) :- Foo(a, b, x), Foo(c, d, y), E(x, y), E(a, c).")) in (
            H.HL_OK, H.HL_E_UNSUPPORTED)
        assert code_of(lambda: e.program("P(a, b) :- Foo(a, b, c).")) == H.HL_E_INVALID
        assert code_of(lambda: e.index("Foo", 0)) == H.HL_E_UNSUPPORTED
    finally:
        e.close()
