"""GPU fixpoints against the oracle, bit-exact: final IDB sets (sorted rows)
and the per-iteration delta and new-tuple counts.  Small inputs that still
span several tiles and ragged tails; edge cases of the method."""

import os
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
        for n in ("reach", "sg", "cspa_shaped")}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_eval(program, edb, idb, **kw):
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    return pkg.evaluate(program, edb, idb, device=0, stream=torch.cuda.current_stream(), **kw)


def check_same(program, edb, idb, **kw):
    want = oracle.evaluate(program, edb, idb, max_iterations=100_000)
    rels, deltas, st = gpu_eval(program, edb, idb, **kw)
    for name in idb:
        assert np.array_equal(rels[name], want.relations[name]), name
        assert deltas[name] == want.deltas[name], name
    return rels, deltas, st, want


def test_reach_er1000():
    say("reach er1000")
    wl = workloads.reach_er_1000()
    rels, deltas, st, want = check_same(PROG["reach"], wl["edb"], {"Reach": 2})
    assert st.key_bytes == 4 and st.id_bits == 10
    assert st.iterations == want.iterations


def test_new_counts_match_oracle():
    import torch
    import paper_2311_02206_amd as pkg
    say("new counts sg tree")
    wl = workloads.scaled_tree(3000, seed=5)
    want = oracle.evaluate(PROG["sg"], wl["edb"], {"SG": 2})
    with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
        e.declare("Edge", 2, True)
        e.declare("SG", 2, False)
        e.load("Edge", wl["edb"]["Edge"])
        e.program(PROG["sg"])
        e.run()
        assert e.iteration_counts("SG", 1) == want.news["SG"]
        assert e.iteration_counts("SG", 0) == want.deltas["SG"]


def test_sg_paper_example():
    say("sg paper example")
    E = np.array([[9, 0], [9, 2], [0, 3], [1, 3], [1, 4], [1, 5], [2, 5], [3, 6], [4, 7], [4, 8],
                  [5, 8], [6, 10], [8, 11], [12, 10], [12, 11]], dtype=np.uint32)
    rels, deltas, st, want = check_same(PROG["sg"], {"Edge": E}, {"SG": 2})
    assert deltas["SG"] == [12, 4, 0]


@pytest.mark.parametrize("n", [2, 50, 2000, 6000])
def test_sg_tree(n):
    say(f"sg tree {n}")
    wl = workloads.scaled_tree(n, seed=n)
    rels, deltas, st, want = check_same(PROG["sg"], wl["edb"], {"SG": 2})
    total, cf = oracle.sg_tree_closed_form(wl["edb"]["Edge"])
    assert len(rels["SG"]) == total and deltas["SG"] == cf


def test_sg_tree_40k_closed_form():
    """Too large for the std::set oracle (~6e8 tuples): closed form only."""
    say("sg tree 40000 (closed form)")
    wl = workloads.scaled_tree(40_000, seed=40_000)
    rels, deltas, st = gpu_eval(PROG["sg"], wl["edb"], {"SG": 2})
    total, cf = oracle.sg_tree_closed_form(wl["edb"]["Edge"])
    assert len(rels["SG"]) == total and deltas["SG"] == cf


@pytest.mark.parametrize("scale,m", [(8, 700), (10, 3000), (12, 12_000)])
def test_reach_rmat_small(scale, m):
    say(f"reach rmat {scale} {m}")
    wl = workloads.scaled_rmat(scale, m, seed=scale)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2})


def test_reach_closed_forms():
    for n in (2, 3, 100, 700):
        say(f"reach closed forms n={n}")
        path = np.array([[i, i + 1] for i in range(n - 1)], dtype=np.uint32)
        rels, deltas, st = gpu_eval(PROG["reach"], {"Edge": path}, {"Reach": 2})
        assert len(rels["Reach"]) == n * (n - 1) // 2
        assert deltas["Reach"] == list(range(n - 1, 0, -1)) + [0]
        cyc = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.uint32)
        rels, _, _ = gpu_eval(PROG["reach"], {"Edge": cyc}, {"Reach": 2})
        assert len(rels["Reach"]) == n * n
    say("reach empty / self loop")
    rels, deltas, st = gpu_eval(PROG["reach"], {"Edge": np.zeros((0, 2), np.uint32)},
                                {"Reach": 2})
    assert len(rels["Reach"]) == 0 and deltas["Reach"] == [0]
    rels, deltas, st = gpu_eval(PROG["reach"], {"Edge": np.array([[7, 7]], np.uint32)},
                                {"Reach": 2})
    assert rels["Reach"].tolist() == [[7, 7]]


def test_wide_ids_use_64bit_keys():
    say("wide ids")
    wl = workloads.reach_er_1000()
    E = wl["edb"]["Edge"].astype(np.uint64)
    # spread ids over the whole uint32 range, including 0 and 2^32-1
    perm = (E * np.uint64(4294967291) + np.uint64(12345)) % np.uint64(1 << 32)
    perm[0, 0] = 0
    perm[1, 1] = 0xFFFFFFFF
    E2 = perm.astype(np.uint32)
    rels, deltas, st, want = check_same(PROG["reach"], {"Edge": E2}, {"Reach": 2})
    assert st.key_bytes == 8 and st.id_bits == 32


def test_duplicates_and_row_order():
    say("duplicates")
    wl = workloads.scaled_rmat(9, 1500, seed=4)
    E = wl["edb"]["Edge"]
    rng = np.random.default_rng(0)
    E2 = np.concatenate([E[rng.permutation(len(E))], E[:300], E[:10]])
    r1, d1, _ = gpu_eval(PROG["reach"], {"Edge": E}, {"Reach": 2})
    r2, d2, _ = gpu_eval(PROG["reach"], {"Edge": E2}, {"Reach": 2})
    assert np.array_equal(r1["Reach"], r2["Reach"]) and d1 == d2


def test_ebm_off_and_arena_give_same_result():
    import torch
    say("ebm off / arena")
    wl = workloads.scaled_rmat(10, 3000, seed=8)
    r0, d0, s0 = gpu_eval(PROG["reach"], wl["edb"], {"Reach": 2})
    r1, d1, s1 = gpu_eval(PROG["reach"], wl["edb"], {"Reach": 2}, ebm=False)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    r2, d2, s2 = gpu_eval(PROG["reach"], wl["edb"], {"Reach": 2}, arena=arena)
    for r, d in ((r1, d1), (r2, d2)):
        assert np.array_equal(r["Reach"], r0["Reach"]) and d == d0
    assert s1.allocations > s0.allocations


def test_two_delta_variants():
    say("two delta variants")
    prog = """P(a, b) :- E(a, b).
P(a, b) :- P(a, c), F(c, b).
Q(a, b) :- P(a, c), P(c, b)."""
    edb = {"E": np.array([[1, 2], [2, 3]], np.uint32),
           "F": np.array([[3, 4], [4, 5], [5, 6]], np.uint32)}
    rels, deltas, st, want = check_same(prog, edb, {"P": 2, "Q": 2})
    assert [1, 4] in rels["Q"].tolist()


def test_nonlinear_closure():
    say("nonlinear closure")
    prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."
    wl = workloads.scaled_rmat(10, 2500, seed=3)
    check_same(prog, {"E": wl["edb"]["Edge"]}, {"T": 2})


def test_random_programs():
    """Random binary-relation programs (the brute-force pin generator): those
    outside the binary chain form (cross products, three live variables) run
    as wide plans; every one must match."""
    import random
    import paper_2311_02206_amd as pkg
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from test_oracle_pins import random_program, render
    rng = random.Random(77)
    ran = 0
    for k in range(120):
        rules = random_program(rng)
        n = rng.randint(3, 40)
        edb = {}
        for name in ("E", "F"):
            m = rng.randint(0, 3 * n)
            edb[name] = np.array(sorted({(rng.randrange(n), rng.randrange(n)) for _ in range(m)}),
                                 dtype=np.uint32).reshape(-1, 2)
        prog = render(rules)
        try:
            check_same(prog, edb, {"P": 2, "Q": 2})
            ran += 1
        except pkg.HlError as e:
            assert e.code == pkg.hisalog.HL_E_UNSUPPORTED, (prog, e)
    say(f"random programs run: {ran}")
    assert ran >= 110


def test_cspa_shaped_small():
    say("cspa small")
    A = workloads.zipf_pairs(1 << 9, 300, 1.2, 0xC3, 0, orient="by_rank")
    D = workloads.zipf_pairs(1 << 9, 120, 1.2, 0xC3, 1, orient="by_rank")
    check_same(PROG["cspa_shaped"], {"Assign": A, "Dereference": D},
               {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2})


@pytest.mark.parametrize("case", ["reach_rmat", "sg_tree", "cspa", "wide", "nonlinear"])
def test_join_dedup_matches_plain(case):
    """Dropping repeated join outputs inside a tile (HL_FLAG_JOIN_DEDUP) must
    not change any result; it only lowers the number of keys sorted."""
    say(f"join dedup on/off: {case}")
    if case == "reach_rmat":
        prog, edb, idb = PROG["reach"], workloads.scaled_rmat(11, 6000, seed=4)["edb"], {"Reach": 2}
    elif case == "sg_tree":
        prog, edb, idb = PROG["sg"], workloads.scaled_tree(3000, seed=3)["edb"], {"SG": 2}
    elif case == "cspa":
        prog, edb = PROG["cspa_shaped"], workloads.cspa(10)["edb"]
        idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    elif case == "wide":
        E = workloads.reach_er_1000()["edb"]["Edge"].astype(np.uint64)
        E = ((E * np.uint64(4294967291) + np.uint64(12345)) % np.uint64(1 << 32)).astype(np.uint32)
        prog, edb, idb = PROG["reach"], {"Edge": E}, {"Reach": 2}
    else:
        prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."
        edb, idb = {"E": workloads.scaled_rmat(10, 2500, seed=3)["edb"]["Edge"]}, {"T": 2}
    rels, deltas, st, want = check_same(prog, edb, idb, join_dedup=True)
    r0, d0, st0 = gpu_eval(prog, edb, idb)
    for n in idb:
        assert np.array_equal(rels[n], r0[n]) and deltas[n] == d0[n]
    assert st.join_outputs == st0.join_outputs
    assert st.candidates <= st.join_outputs
    assert st0.candidates <= st0.join_outputs
    if case in ("reach_rmat", "cspa", "nonlinear"):
        assert st.candidates < st0.candidates  # duplicates were dropped


@pytest.mark.parametrize("case", ["reach_rmat", "sg_tree", "cspa"])
def test_autotune_keeps_results(case):
    """The autotuner times alternative settings; whichever it keeps, the
    relations it leaves and every later run equal the oracle's."""
    import torch
    import paper_2311_02206_amd as pkg
    say(f"autotune: {case}")
    if case == "reach_rmat":
        prog, edb, idb = PROG["reach"], workloads.scaled_rmat(11, 6000, seed=4)["edb"], {"Reach": 2}
    elif case == "sg_tree":
        prog, edb, idb = PROG["sg"], workloads.scaled_tree(3000, seed=3)["edb"], {"SG": 2}
    else:
        prog, edb = PROG["cspa_shaped"], workloads.cspa(10)["edb"]
        idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    want = oracle.evaluate(prog, edb, idb)
    with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
        for n in edb:
            e.declare(n, 2, True)
        for n in idb:
            e.declare(n, 2, False)
        for n, rows in edb.items():
            e.load(n, rows)
        e.program(prog)
        t = e.autotune(reps=1)
        say(f"  chose {t}")
        assert t["trials"] >= 4 and t["best_seconds"] <= t["first_seconds"]
        assert t["hash_load_factor"] in (0.5, 0.8) and t["ebm_k"] in (1.5, 8.0)
        assert t["sort_tile"] in (4096, 8192) and t["diff_tile"] in (2048, 4096)
        for _ in range(2):
            for n in idb:
                assert np.array_equal(e.fetch(n), want.relations[n]), n
                assert e.iteration_counts(n, 0) == want.deltas[n], n
            e.run()


@pytest.mark.parametrize("learned", [False, True])
def test_cspa_literal_2p11(learned):
    """The CSPA-shaped program on the literal Zipf reading at 2^11 ids (781
    Assign, 292 Dereference pairs): the largest size the std::set oracle
    finishes in seconds."""
    say(f"cspa literal 2^11, learned={learned}")
    wl = workloads.cspa(11)
    check_same(PROG["cspa_shaped"], wl["edb"],
               {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}, learned=learned)


@pytest.mark.parametrize("case", ["reach_er1000", "sg_tree", "cspa", "wide", "nonlinear"])
def test_learned_index_matches_plain(case):
    """The learned position index replaces the hash probe and the membership
    search; results must not change (and must match the oracle)."""
    say(f"learned vs plain: {case}")
    if case == "reach_er1000":
        prog, edb, idb = PROG["reach"], workloads.reach_er_1000()["edb"], {"Reach": 2}
    elif case == "sg_tree":
        prog, edb, idb = PROG["sg"], workloads.scaled_tree(3000, seed=3)["edb"], {"SG": 2}
    elif case == "cspa":
        prog = PROG["cspa_shaped"]
        edb = {"Assign": workloads.zipf_pairs(1 << 9, 300, 1.2, 0xC3, 0, orient="by_rank"),
               "Dereference": workloads.zipf_pairs(1 << 9, 120, 1.2, 0xC3, 1, orient="by_rank")}
        idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    elif case == "wide":
        E = workloads.reach_er_1000()["edb"]["Edge"].astype(np.uint64)
        E = ((E * np.uint64(4294967291) + np.uint64(12345)) % np.uint64(1 << 32)).astype(np.uint32)
        prog, edb, idb = PROG["reach"], {"Edge": E}, {"Reach": 2}
    else:
        prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."
        edb, idb = {"E": workloads.scaled_rmat(10, 2500, seed=3)["edb"]["Edge"]}, {"T": 2}
    rels, deltas, st, want = check_same(prog, edb, idb, learned=True)
    r0, d0, _ = gpu_eval(prog, edb, idb)
    for n in idb:
        assert np.array_equal(rels[n], r0[n]) and deltas[n] == d0[n]


@pytest.mark.parametrize("learned", [False, True])
def test_chunked_new_tuples(learned):
    """An iteration's new tuples beyond one sort chunk (forced here to 4,096
    keys), and a single join's outputs beyond one chunk, are processed chunk
    by chunk into a pending delta; results must not change.  Covers an
    unfiltered join (Reach), filtered ones (SG), several rules deriving one
    relation and a three-atom rule (CSPA-shaped), and in-tile dedup."""
    say(f"chunked sort, learned={learned}")
    wl = workloads.scaled_rmat(10, 3000, seed=8)
    rels, deltas, st, want = check_same(PROG["reach"], wl["edb"], {"Reach": 2},
                                        sort_chunk_log2=12, learned=learned)
    assert st.candidates > 50 * 4096
    wl = workloads.scaled_tree(2000, seed=2)
    check_same(PROG["sg"], wl["edb"], {"SG": 2}, sort_chunk_log2=12, learned=learned)
    cs = workloads.cspa(10)["edb"]
    idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    check_same(PROG["cspa_shaped"], cs, idb, sort_chunk_log2=12, learned=learned)
    check_same(PROG["cspa_shaped"], cs, idb, sort_chunk_log2=12, learned=learned,
               join_dedup=True)
    wl = workloads.scaled_rmat(10, 3000, seed=8)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2}, sort_chunk_log2=13, learned=learned,
               join_dedup=True)


def test_memory_budget():
    """Under a device budget the engine returns cached blocks to the device
    before exceeding it and still computes the fixpoint exactly; a budget
    too small fails with HL_E_NOMEM and leaves the engine usable."""
    import torch
    import paper_2311_02206_amd as pkg
    say("memory budget")
    wl = workloads.scaled_rmat(11, 6000, seed=4)
    want = oracle.evaluate(PROG["reach"], wl["edb"], {"Reach": 2})

    def make(budget):
        e = pkg.Engine(device=0, stream=torch.cuda.current_stream(), budget_bytes=budget)
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.load("Edge", wl["edb"]["Edge"])
        e.program(PROG["reach"])
        return e

    with make(0) as e:
        peak = e.run().peak_bytes
    with make(int(peak * 1.3)) as e:
        for _ in range(3):
            st = e.run()
            assert st.peak_bytes <= int(peak * 1.3)
            assert np.array_equal(e.fetch("Reach"), want.relations["Reach"])
            assert e.iteration_counts("Reach", 0) == want.deltas["Reach"]
    with make(peak // 8) as e:
        with pytest.raises(pkg.HlError) as ei:
            e.run()
        assert ei.value.code == pkg.hisalog.HL_E_NOMEM
        with pytest.raises(pkg.HlError):
            e.run()
    with make(int(peak * 1.3)) as e:  # a fresh engine on the same device works
        e.run()
        assert np.array_equal(e.fetch("Reach"), want.relations["Reach"])


def test_error_paths():
    import torch
    import paper_2311_02206_amd as pkg
    say("error paths")
    with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
        e.declare("E", 2, True)
        e.declare("R", 2, False)
        with pytest.raises(pkg.HlError) as ei:
            e.declare("E", 2, True)
        assert ei.value.code == pkg.hisalog.HL_E_INVALID
        with pytest.raises(pkg.HlError) as ei:
            e.declare("T5", 5, False)
        assert ei.value.code == pkg.hisalog.HL_E_UNSUPPORTED
        with pytest.raises(pkg.HlError) as ei:
            # five filters at one join
            e.program("R(x, y) :- E(x, a), E(a, y), x != y, x != a, a != y, y != x, a != x.")
        assert ei.value.code == pkg.hisalog.HL_E_UNSUPPORTED
        with pytest.raises(pkg.HlError) as ei:
            e.program("R(x, y) :- E(x, .")
        assert ei.value.code == pkg.hisalog.HL_E_INVALID
        with pytest.raises(pkg.HlError) as ei:
            e.run()  # no program yet
        assert ei.value.code == pkg.hisalog.HL_E_STATE
        e.program("R(x, y) :- E(x, y).\nR(x, y) :- E(x, z), R(z, y).\nR(x, x) :- E(x, y), E(y, x).")
        e.load("E", np.array([[1, 2], [2, 3]], np.uint32))
        e.run()
        import ctypes
        n = ctypes.c_uint64()
        rc = e._L.hl_fetch(e._h, b"R", None, 0, ctypes.byref(n))
        assert rc == pkg.hisalog.HL_E_CAPACITY and n.value == 3
        assert e.fetch("R").tolist() == [[1, 2], [1, 3], [2, 3]]
        e.load("E", np.array([[2, 1]], np.uint32))
        e.run()
        assert e.fetch("R").tolist() == [[1, 1], [1, 2], [1, 3], [2, 1], [2, 2], [2, 3]]
    say("budget exhaustion")
    wl = workloads.scaled_rmat(10, 3000, seed=8)
    with pytest.raises(pkg.HlError) as ei:
        gpu_eval(PROG["reach"], wl["edb"], {"Reach": 2}, budget_bytes=1 << 16)
    assert ei.value.code == pkg.hisalog.HL_E_NOMEM


@pytest.mark.parametrize("case", ["sg_paper", "sg_tree", "sg_tree_learned", "cspa", "random"])
def test_nested_joins_match_oracle(case):
    """The nested evaluation of two-join bodies (the Section 5.2 ablation)
    gives the oracle's result: same-generation (a filter on the second
    join), the CSPA-shaped program (a three-atom rule among two-atom ones)
    and random two- and three-atom programs."""
    say(f"nested joins, {case}")
    if case == "sg_paper":
        E = np.array([[9, 0], [9, 2], [0, 3], [1, 3], [1, 4], [1, 5], [2, 5], [3, 6], [4, 7],
                      [4, 8], [5, 8], [6, 10], [8, 11], [12, 10], [12, 11]], dtype=np.uint32)
        check_same(PROG["sg"], {"Edge": E}, {"SG": 2}, nested_joins=True)
    elif case.startswith("sg_tree"):
        wl = workloads.scaled_tree(3000, seed=23)
        check_same(PROG["sg"], wl["edb"], {"SG": 2}, nested_joins=True,
                   learned=case.endswith("learned"))
    elif case == "cspa":
        cs = workloads.cspa(11)["edb"]
        check_same(PROG["cspa_shaped"], cs, {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2},
                   nested_joins=True)
    else:
        rng = np.random.default_rng(29)
        progs = ["P(x, y) :- E(x, y).\nP(x, y) :- E(x, a), P(a, b), F(b, y), x != y.\n",
                 "P(x, y) :- F(y, x).\nP(x, y) :- P(x, a), E(a, b), E(b, y).\n",
                 "P(x, y) :- E(x, y).\nP(x, y) :- E(a, x), P(a, b), E(y, b).\n"]
        for prog in progs:
            E = rng.integers(0, 40, size=(120, 2)).astype(np.uint32)
            F = rng.integers(0, 40, size=(60, 2)).astype(np.uint32)
            check_same(prog, {"E": E, "F": F}, {"P": 2}, nested_joins=True)


@pytest.mark.parametrize("tile", [1024, 4096])
def test_expand_tiles_match_oracle(tile):
    """Join expand tiles of 1,024 and 4,096 outputs (2,048 is the default
    everywhere else): plain, with in-tile dedup (its LDS set scales with the
    tile), and with joins expanded a range of tiles at a time."""
    say(f"expand tile {tile}")
    wl = workloads.scaled_rmat(12, 12_000, seed=0xC2A)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2}, expand_tile=tile)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2}, expand_tile=tile, join_dedup=True)
    tr = workloads.scaled_tree(2000, seed=31)
    check_same(PROG["sg"], tr["edb"], {"SG": 2}, expand_tile=tile, sort_chunk_log2=12)
    cs = workloads.cspa(11)["edb"]
    check_same(PROG["cspa_shaped"], cs, {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2},
               expand_tile=tile, join_dedup=True)


@pytest.mark.parametrize("sort_tile,diff_tile", [(4096, 2048), (4096, 4096), (8192, 2048)])
def test_sort_and_difference_tiles_match_oracle(sort_tile, diff_tile):
    """Radix sort tiles of 4,096 keys and set difference tiles of 2,048
    candidates (8,192 and 4,096 are the defaults everywhere else), with
    32- and 64-bit keys, chunked sorts and the learned index's windows."""
    say(f"sort tile {sort_tile}, difference tile {diff_tile}")
    kw = dict(sort_tile=sort_tile, diff_tile=diff_tile)
    wl = workloads.scaled_rmat(12, 12_000, seed=0xC2A)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2}, **kw)
    check_same(PROG["reach"], wl["edb"], {"Reach": 2}, learned=True, sort_chunk_log2=14, **kw)
    tr = workloads.scaled_tree(2000, seed=31)
    check_same(PROG["sg"], tr["edb"], {"SG": 2}, **kw)
    E = workloads.reach_er_1000()["edb"]["Edge"].astype(np.uint64)
    E = ((E * np.uint64(4294967291) + np.uint64(12345)) % np.uint64(1 << 32)).astype(np.uint32)
    check_same(PROG["reach"], {"Edge": E}, {"Reach": 2}, **kw)


UNARY = ("R(x) :- S(x).\nR(y) :- R(x), E(x, y).\nN(x) :- E(x, _).\nN(y) :- E(_, y).\n"
         "B(x, y) :- R(x), E(y, x), x != y.\nL(x) :- E(x, x).\nC(x, x) :- R(x), L(x).\n")
UNARY_IDB = {"R": 1, "N": 1, "B": 2, "L": 1, "C": 2}
# the part that fused iterations take (every join inner an EDB relation)
UNARY_FUSED = "R(x) :- S(x).\nR(y) :- R(x), E(x, y).\nB(x, y) :- R(x), E(y, x), x != y.\n"


@pytest.mark.parametrize("mode", ["plain", "learned", "fused_graph"])
def test_unary_relations(mode):
    """Unary EDB and IDB relations against the oracle: single-source
    reachability (pinned to BFS), projections, a unary atom as a join's
    outer and inner, a self-loop test and a binary head over a unary body."""
    say(f"unary relations, {mode}")
    kw = {"plain": {}, "learned": {"learned": True},
          "fused_graph": {"fused": True, "hip_graph": True}}[mode]
    wl = workloads.reach_er_1000()
    E = np.concatenate([wl["edb"]["Edge"], np.array([[7, 7], [500, 500]], dtype=np.uint32)])
    S = np.array([[0], [17], [999]], dtype=np.uint32)
    edb = {"E": E, "S": S}
    if mode == "fused_graph":
        rels, deltas, st, want = check_same(UNARY_FUSED, edb, {"R": 1, "B": 2}, **kw)
    else:
        rels, deltas, st, want = check_same(UNARY, edb, UNARY_IDB, **kw)
    reach = set()
    for s in (0, 17, 999):
        reach |= {s} | set(oracle.reach_from(wl["n_nodes"], E, s).tolist())
    assert sorted(reach) == rels["R"][:, 0].tolist()
    assert rels["R"].shape[1] == 1 and rels["B"].shape[1] == 2
    if mode == "fused_graph":
        assert st.fused_iterations > 0


def test_rule_stats_closed_forms():
    """Per-rule join outputs (hl_rule_stats) against counts that follow from
    the final relations: every Reach tuple (z, y) lies in exactly one delta
    and joins the in-edges of z once; the first same-generation rule yields
    sum_p outdeg(p)^2 outputs before its filter, and every SG tuple (a, b)
    lies in one delta and yields outdeg(a) first-join and
    outdeg(a) * outdeg(b) last-join outputs.  The rules' outputs add up to
    the run's join outputs."""
    import torch
    import paper_2311_02206_amd as pkg
    say("rule stats: reach er1000, sg tree")
    E = np.unique(workloads.reach_er_1000()["edb"]["Edge"], axis=0)
    T = workloads.scaled_tree(3000, seed=3)["edb"]["Edge"]
    for prog, edb, idb in ((PROG["reach"], {"Edge": E}, "Reach"),
                           (PROG["sg"], {"Edge": T}, "SG")):
        with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
            e.declare("Edge", 2, True)
            e.declare(idb, 2, False)
            e.load("Edge", edb["Edge"])
            e.program(prog)
            st = e.run()
            R = e.fetch(idb).astype(np.int64)
            rs = e.rule_stats()
        assert len(rs) == 2
        assert sum(o for o, _ in rs) == st.join_outputs
        G = edb["Edge"].astype(np.int64)
        n = int(max(G.max(), R.max() if len(R) else 0)) + 1
        if idb == "Reach":
            indeg = np.bincount(G[:, 1], minlength=n)
            assert rs[0] == (len(G), 0)
            assert rs[1] == (int(indeg[R[:, 0]].sum()), 0)
        else:
            outdeg = np.bincount(G[:, 0], minlength=n)
            assert rs[0] == (int((outdeg ** 2).sum()), 0)
            assert rs[1] == (int((outdeg[R[:, 0]] * outdeg[R[:, 1]]).sum()),
                             int(outdeg[R[:, 0]].sum()))


@pytest.mark.parametrize("learned", [False, True])
@pytest.mark.parametrize("case", ["nonlinear", "cspa", "reach", "sg"])
def test_tail_runs_and_levels_match_oracle(case, learned):
    """Tail runs forced at small sizes (tail_min_bytes 1): relations probed as
    join inners kept as two levels (the nonlinear closure probes both
    columns of its own relation; CSPA's three mutually recursive relations),
    relations no join probes with a plain tail run (Reach, SG), with hash and
    learned probes, chunked new tuples (absorbed chunk by chunk against full
    and the tail), and the same with levels off."""
    say(f"tails and levels: {case}, learned={learned}")
    if case == "nonlinear":
        prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."
        edb, idb = {"E": workloads.scaled_rmat(10, 2500, seed=3)["edb"]["Edge"]}, {"T": 2}
    elif case == "cspa":
        prog, edb = PROG["cspa_shaped"], workloads.cspa(10)["edb"]
        idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    elif case == "reach":
        prog, edb, idb = PROG["reach"], workloads.scaled_rmat(11, 6000, seed=4)["edb"], {"Reach": 2}
    else:
        prog, edb, idb = PROG["sg"], workloads.scaled_tree(3000, seed=3)["edb"], {"SG": 2}
    want = oracle.evaluate(prog, edb, idb, max_iterations=100_000)
    for kw in ({}, {"sort_chunk_log2": 12}, {"levels": False}):
        rels, deltas, st = gpu_eval(prog, edb, idb, learned=learned, tail_min_bytes=1, **kw)
        for name in idb:
            assert np.array_equal(rels[name], want.relations[name]), (name, kw)
            assert deltas[name] == want.deltas[name], (name, kw)


@pytest.mark.parametrize("case", ["reach", "sg", "cspa", "wide"])
def test_outer_slices_match_oracle(case):
    """A join's outer side taken 256 tuples at a time (outer_slice_log2 8;
    2^28 is the default): Reach, same-generation's three-atom rule (whose
    intermediate result is built per slice), the CSPA-shaped program, a
    wide program, nested joins, chunked new tuples and two-level inners."""
    say(f"outer slices: {case}")
    kw = dict(outer_slice_log2=8)
    if case == "reach":
        prog, edb, idb = PROG["reach"], workloads.scaled_rmat(11, 6000, seed=4)["edb"], {"Reach": 2}
        extra = ({"sort_chunk_log2": 12}, {"learned": True})
    elif case == "sg":
        prog, edb, idb = PROG["sg"], workloads.scaled_tree(3000, seed=3)["edb"], {"SG": 2}
        extra = ({"nested_joins": True}, {"sort_chunk_log2": 12})
    elif case == "cspa":
        prog, edb = PROG["cspa_shaped"], workloads.cspa(10)["edb"]
        idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
        extra = ({"tail_min_bytes": 1}, {"learned": True, "tail_min_bytes": 1})
    else:
        rng = np.random.default_rng(7)
        E = np.stack([rng.integers(0, 300, 900), rng.integers(0, 300, 900),
                      rng.integers(0, 3, 900)], 1).astype(np.uint32)
        prog = "P(x, y, l) :- E(x, y, l).\nP(x, z, l) :- P(x, y, l), E(y, z, l)."
        edb, idb = {"E": E}, {"P": 3}
        extra = ({"learned": True},)
    want = oracle.evaluate(prog, edb, idb, max_iterations=100_000)
    for more in ({},) + extra:
        rels, deltas, st = gpu_eval(prog, edb, idb, **kw, **more)
        for name in idb:
            assert np.array_equal(rels[name], want.relations[name]), (name, more)
            assert deltas[name] == want.deltas[name], (name, more)
