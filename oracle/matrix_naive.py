"""Naive Datalog evaluation over binary relations as boolean matrix products.

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

What it computes: the least model of a positive program, the least fixpoint
of the immediate-consequence operator T_P (Section 2, Datalog background),
reached by naive iteration from the empty IDB:

    full_0 = {},  full_{i+1} = full_i  union  T_P(full_i)

with every rule evaluated against the whole of ``full_i`` (Jacobi: all
rules see the same state).  The per-iteration increments
``full_{i+1} - full_i`` are exactly the delta sizes a Jacobi semi-naive
evaluator produces (Section 2, semi-naive evaluation): a derivation that
uses no new tuple was already made one iteration earlier.

How a rule is evaluated: each relation over the ids that occur in the EDB is
a 0/1 matrix (every IDB id comes from some EDB tuple, since each head
variable is bound by a body atom).  A rule body is a conjunction, so its
result is an existential projection onto the head variables; variables that
are not in the head are eliminated one at a time, each by a matrix product
(two atoms share the variable), a masked reduction (one atom) or an
element-wise conjunction.  Products are taken in float32 with a ``> 0``
test; the sums are integers below 2^24 for every size used here, so they
are exact.

This is a second algorithm, independent of the std::set evaluator in
``semi_naive.cpp`` (its own parser, no tuple sets, no semi-naive deltas);
it serves where the std::set evaluator would take hours (millions of
output tuples, tens of billions of duplicate derivations).

Supported: binary relations, atoms with variables or the wildcard ``_``,
filters ``x != y`` between body variables (each one a conjunct whose
matrix is the complement of the identity), bodies where each eliminated
variable occurs in at most two two-variable conjuncts at its turn.  Anything
else raises ``NotImplementedError``.
"""

from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np

_ATOM = re.compile(r"\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(([^()]*)\)\s*")
_NEQ = re.compile(r"\s*([A-Za-z_][A-Za-z0-9_]*)\s*!=\s*([A-Za-z_][A-Za-z0-9_]*)\s*$")


@dataclass
class Rule:
    head: tuple            # (relation, (var, var))
    atoms: list            # [(relation, (arg, arg))], arg a name or "_"
    neq: list              # [(var, var)]


@dataclass
class MatrixResult:
    relations: dict = field(default_factory=dict)   # name -> sorted (n, 2) uint32
    deltas: dict = field(default_factory=dict)      # name -> per-iteration counts
    iterations: int = 0
    active_ids: int = 0


def _strip_comments(text: str) -> str:
    out = []
    for line in text.splitlines():
        for mark in ("//", "#"):
            k = line.find(mark)
            if k >= 0:
                line = line[:k]
        out.append(line)
    return "\n".join(out)


def _split_top(body: str) -> list:
    """Split a rule body at the commas that are outside parentheses."""
    parts, depth, cur = [], 0, []
    for ch in body:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == "," and depth == 0:
            parts.append("".join(cur))
            cur = []
        else:
            cur.append(ch)
    parts.append("".join(cur))
    return [p for p in (q.strip() for q in parts) if p]


def parse(text: str) -> list:
    rules = []
    for stmt in _strip_comments(text).split("."):
        if not stmt.strip():
            continue
        if ":-" not in stmt:
            raise NotImplementedError(f"not a rule: {stmt.strip()!r}")
        head_s, body_s = stmt.split(":-", 1)
        m = _ATOM.fullmatch(head_s)
        if not m:
            raise NotImplementedError(f"bad head {head_s!r}")
        hargs = tuple(a.strip() for a in m.group(2).split(","))
        if len(hargs) != 2 or "_" in hargs:
            raise NotImplementedError(f"head must have two variables: {head_s!r}")
        atoms, neq = [], []
        for part in _split_top(body_s):
            f = _NEQ.fullmatch(part)
            if f:
                neq.append((f.group(1), f.group(2)))
                continue
            a = _ATOM.fullmatch(part)
            if not a:
                raise NotImplementedError(f"bad body element {part!r}")
            args = tuple(x.strip() for x in a.group(2).split(","))
            if len(args) != 2:
                raise NotImplementedError(f"only binary atoms: {part!r}")
            atoms.append((a.group(1), args))
        rules.append(Rule((m.group(1), hargs), atoms, neq))
    return rules


def _bool_product(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(a @ b) > 0 for 0/1 matrices: exact while inner sizes stay < 2^24."""
    assert a.shape[1] < (1 << 24)
    return (a.astype(np.float32) @ b.astype(np.float32)) > 0


class _Factor:
    """A conjunct over one or two variables (or none: a truth value)."""

    def __init__(self, vars_, arr):
        self.vars = tuple(vars_)
        self.arr = arr

    def oriented(self, first):
        """The matrix with ``first`` as its row variable."""
        if self.vars[0] == first:
            return self.arr
        return self.arr.T


def _atom_factor(args, mat):
    a, b = args
    if a == "_" and b == "_":
        return _Factor((), np.array(mat.any()))
    if a == "_":
        return _Factor((b,), mat.any(axis=0))
    if b == "_":
        return _Factor((a,), mat.any(axis=1))
    if a == b:
        return _Factor((a,), np.diagonal(mat).copy())
    return _Factor((a, b), mat)


def _merge_same_vars(factors):
    """Conjoin factors over the same variable set into one."""
    by = {}
    for f in factors:
        key = frozenset(f.vars)
        if key in by:
            g = by[key]
            if len(g.vars) == 2:
                g.arr = g.arr & f.oriented(g.vars[0])
            else:
                g.arr = g.arr & f.arr
        else:
            by[key] = _Factor(f.vars, f.arr.copy())
    return list(by.values())


def _eliminate(factors, z):
    """Existentially project variable ``z`` out of the conjunction."""
    with_z = [f for f in factors if z in f.vars]
    rest = [f for f in factors if z not in f.vars]
    mask = None
    mats = []
    for f in with_z:
        if len(f.vars) == 1:
            mask = f.arr if mask is None else (mask & f.arr)
        else:
            mats.append(f)
    if len(mats) > 2:
        return None
    if not mats:
        rest.append(_Factor((), np.array(mask.any())))
        return rest
    if mask is not None:
        m0 = mats[0].oriented(z) & mask[:, None]
    else:
        m0 = mats[0].oriented(z)
    u = [v for v in mats[0].vars if v != z][0]
    if len(mats) == 1:
        rest.append(_Factor((u,), m0.any(axis=0)))
        return rest
    m1 = mats[1].oriented(z)
    w = [v for v in mats[1].vars if v != z][0]
    if u == w:
        rest.append(_Factor((u,), (m0 & m1).any(axis=0)))
    else:
        rest.append(_Factor((u, w), _bool_product(m0.T, m1)))
    return rest


def _eval_rule(rule, mats, k):
    factors = [_atom_factor(args, mats[name]) for name, args in rule.atoms]
    hx, hy = rule.head[1]
    head_vars = {hx, hy}
    body_vars = {v for f in factors for v in f.vars}
    for a, b in rule.neq:
        if a not in body_vars or b not in body_vars:
            raise NotImplementedError("a filter on a variable the body does not bind")
        if a == b:
            return np.zeros((k, k), dtype=bool)
        # x != y is one more conjunct: the complement of the identity
        factors.append(_Factor((a, b), ~np.eye(k, dtype=bool)))
    while True:
        factors = _merge_same_vars(factors)
        others = sorted({v for f in factors for v in f.vars} - head_vars)
        if not others:
            break
        for z in others:
            out = _eliminate(factors, z)
            if out is not None:
                factors = out
                break
        else:
            raise NotImplementedError("no variable can be eliminated pairwise")
    res = np.ones((k, k), dtype=bool)
    present = set()
    for f in factors:
        if len(f.vars) == 0:
            if not bool(f.arr):
                return np.zeros((k, k), dtype=bool)
        elif len(f.vars) == 1:
            v = f.vars[0]
            present.add(v)
            if hx == hy:
                res &= np.diag(f.arr)
            else:
                res &= (f.arr[:, None] if v == hx else f.arr[None, :])
        else:
            present.update(f.vars)
            res &= f.oriented(hx)
    if head_vars - present:
        raise NotImplementedError("a head variable not bound by the body")
    if hx == hy:
        res &= np.eye(k, dtype=bool)
    return res


def evaluate(program: str, edb: dict, idb: dict, max_iterations: int = 0) -> MatrixResult:
    """Naive Jacobi evaluation of ``program`` (binary relations only).

    ``edb`` maps names to row-major uint32 ``(n, 2)`` arrays; ``idb`` maps
    names to their arity (2).  Returns the sorted, deduplicated IDB
    relations and per-iteration delta counts in the std::set evaluator's
    format: iteration 0 holds the EDB-only rules' tuples and the last
    iteration is the empty one.
    """
    rules = parse(program)
    for name, ar in idb.items():
        if ar != 2:
            raise NotImplementedError("binary relations only")
    vals = [np.asarray(r, dtype=np.uint32).reshape(-1, 2) for r in edb.values()]
    ids = np.unique(np.concatenate([v.ravel() for v in vals])) if vals else \
        np.zeros(0, dtype=np.uint32)
    k = len(ids)
    mats = {}
    for name, rows in edb.items():
        rows = np.asarray(rows, dtype=np.uint32).reshape(-1, 2)
        m = np.zeros((k, k), dtype=bool)
        m[np.searchsorted(ids, rows[:, 0]), np.searchsorted(ids, rows[:, 1])] = True
        mats[name] = m
    full = {name: np.zeros((k, k), dtype=bool) for name in idb}
    res = MatrixResult(active_ids=k)
    res.deltas = {name: [] for name in idb}
    it = 0
    while True:
        state = dict(mats)
        state.update(full)
        new = {name: np.zeros((k, k), dtype=bool) for name in idb}
        for rule in rules:
            hname = rule.head[0]
            if hname not in idb:
                raise NotImplementedError(f"rule head {hname} is not an IDB relation")
            new[hname] |= _eval_rule(rule, state, k)
        grown = 0
        for name in idb:
            delta = new[name] & ~full[name]
            c = int(delta.sum())
            res.deltas[name].append(c)
            grown += c
            full[name] |= delta
        it += 1
        if grown == 0 or (max_iterations and it >= max_iterations):
            break
    res.iterations = it
    for name in idb:
        r, c = np.nonzero(full[name])
        res.relations[name] = np.stack([ids[r], ids[c]], axis=1).astype(np.uint32) \
            if len(r) else np.zeros((0, 2), dtype=np.uint32)
    return res
