"""Pins of the oracle on relations of arity 1 to 4 (the paper's requirement
R3, multiple join columns, Section 3; joins on several columns, Section
5.1): random positive programs over EDB relations of arity 3, 2 and 1 and
IDB relations of arity 3, 2 and 4, against the least fixpoint computed by
brute force (the immediate-consequence operator applied over every
assignment of the active domain until nothing changes), final sets and
per-iteration delta sizes both.  The same generator feeds the GPU parity
test of wide programs (test_gpu_wide.py)."""

import itertools
import random

import numpy as np
import pytest

import oracle

ARITY = {"E": 3, "F": 2, "G": 1, "P": 3, "Q": 2, "S": 4}
EDBS = ("E", "F", "G")
IDBS = ("P", "Q", "S")
VARS = "abcde"


def random_wide_program(rng):
    rules = []
    for _ in range(rng.randint(2, 4)):
        body = []
        for _ in range(rng.randint(1, 3)):
            r = rng.choice(list(ARITY))
            body.append((r, tuple(rng.choice(VARS) for _ in range(ARITY[r]))))
        bvars = sorted({v for _, args in body for v in args})
        h = rng.choice(IDBS)
        head = (h, tuple(rng.choice(bvars) for _ in range(ARITY[h])))
        filt = tuple(rng.sample(bvars, 2)) if len(bvars) >= 2 and rng.random() < 0.3 else None
        rules.append((head, body, filt))
    # something seeds the IDB relations
    rules.append((("P", ("a", "b", "c")), [("E", ("a", "b", "c"))], None))
    rules.append((("Q", ("a", "b")), [("F", ("a", "b"))], None))
    return rules


def render(rules):
    lines = []
    for head, body, filt in rules:
        parts = [f"{r}({', '.join(args)})" for r, args in body]
        if filt:
            parts.append(f"{filt[0]} != {filt[1]}")
        lines.append(f"{head[0]}({', '.join(head[1])}) :- " + ", ".join(parts) + ".")
    return "\n".join(lines)


def random_wide_edb(rng, n_ids=None):
    n = n_ids or rng.randint(2, 4)
    out = {}
    for r in EDBS:
        m = rng.randint(0, 6)
        out[r] = {tuple(rng.randrange(n) for _ in range(ARITY[r])) for _ in range(m)}
    return out


def brute_force(rules, edb):
    """Least fixpoint by applying the rules to every assignment of the
    active domain, round after round.  Returns (final sets, per-round
    delta sizes)."""
    dom = sorted({x for rows in edb.values() for t in rows for x in t})
    full = {r: set() for r in IDBS}
    rel = lambda r: edb[r] if r in edb else full[r]
    deltas = {r: [] for r in IDBS}
    while True:
        fresh = {r: set() for r in IDBS}
        for head, body, filt in rules:
            vs = sorted({v for _, args in body for v in args})
            for vals in itertools.product(dom, repeat=len(vs)):
                b = dict(zip(vs, vals))
                if all(tuple(b[v] for v in args) in rel(r) for r, args in body):
                    if filt and b[filt[0]] == b[filt[1]]:
                        continue
                    fresh[head[0]].add(tuple(b[v] for v in head[1]))
        total = 0
        for r in IDBS:
            d = fresh[r] - full[r]
            deltas[r].append(len(d))
            total += len(d)
        for r in IDBS:
            full[r] |= fresh[r]
        if total == 0:
            return full, deltas


def as_arrays(edb):
    return {r: np.array(sorted(v), dtype=np.uint32).reshape(-1, ARITY[r]) for r, v in edb.items()}


def run_oracle(rules, edb, plant=0):
    return oracle.evaluate(render(rules), as_arrays(edb), {r: ARITY[r] for r in IDBS},
                           plant=plant, max_iterations=200)


def wide_cases(n=120, seed=4321):
    rng = random.Random(seed)
    return [(random_wide_program(rng), random_wide_edb(rng)) for _ in range(n)]


CASES = wide_cases()


def as_set(a):
    return {tuple(int(x) for x in row) for row in a}


def test_wide_oracle_matches_brute_force():
    for rules, edb in CASES:
        want, wdeltas = brute_force(rules, edb)
        res = run_oracle(rules, edb)
        for r in IDBS:
            assert as_set(res.relations[r]) == want[r], render(rules)
            assert res.deltas[r] == wdeltas[r], render(rules)


@pytest.mark.parametrize("plant", [1, 3, 5, 6])
def test_wide_pins_catch_planted_mistakes(plant):
    """The oracle with a planted mistake (only the first delta variant; the
    filter's sense inverted; the last tuple of each index range skipped; no
    subtraction of full) must fail the brute-force pin on some of these
    programs."""
    caught = 0
    for rules, edb in CASES:
        want, wdeltas = brute_force(rules, edb)
        try:
            res = run_oracle(rules, edb, plant=plant)
        except RuntimeError:  # never converges (no subtraction of full)
            caught += 1
            continue
        caught += any(as_set(res.relations[r]) != want[r] or res.deltas[r] != wdeltas[r]
                      for r in IDBS)
    assert caught > 0


def test_two_column_join_closed_form():
    """Same-label reachability, P(x, z, l) :- P(x, y, l), E(y, z, l): its
    join key is the two columns (y, l).  Per label, P is the transitive
    closure of that label's edges (scipy's shortest paths)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(3)
    n, labels = 40, 3
    E = np.unique(np.stack([rng.integers(0, n, 150), rng.integers(0, n, 150),
                            rng.integers(0, labels, 150)], 1).astype(np.uint32), axis=0)
    prog = "P(x, y, l) :- E(x, y, l).\nP(x, z, l) :- P(x, y, l), E(y, z, l)."
    res = oracle.evaluate(prog, {"E": E}, {"P": 3})
    want = set()
    for l in range(labels):
        el = E[E[:, 2] == l]
        if len(el) == 0:
            continue
        A = csr_matrix((np.ones(len(el)), (el[:, 0], el[:, 1])), shape=(n, n))
        D = shortest_path(A, unweighted=True, directed=True)
        for s in range(n):
            for t in range(n):
                if s != t:
                    if np.isfinite(D[s, t]):
                        want.add((s, t, l))
                elif A[s, s] or any(u != s and np.isfinite(D[s, u]) and np.isfinite(D[u, s])
                                    for u in range(n)):
                    want.add((s, s, l))  # s lies on a cycle of label l
    assert as_set(res.relations["P"]) == want
