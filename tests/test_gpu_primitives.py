"""GPU parity of each kernel of an iteration against plain numpy definitions:
sort (Section 4.2 / Algorithm 1), unique + set difference (Section 5.1,
populating delta), merge (Section 4.2, merge path) and the HISA range
query (Section 4.3 / Algorithm 2).  Bit-exact."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U = {4: np.uint32, 8: np.uint64}
S = {4: np.int32, 8: np.int64}


@pytest.fixture(scope="module")
def eng():
    import torch
    import paper_2311_02206_amd as pkg
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    e = pkg.Engine(device=0, stream=torch.cuda.current_stream())
    yield e
    e.close()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, kb):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U[kb]).view(S[kb])).cuda()


def to_host(t, kb):
    return t.cpu().numpy().view(U[kb])


def rand_keys(rng, n, kb, bits):
    hi = (1 << bits) - 1
    if kb == 8:
        a = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=n, dtype=np.uint64)
        return a & np.uint64(hi)
    return (rng.integers(0, 1 << 32, size=n, dtype=np.uint64) & np.uint64(hi)).astype(np.uint32)


SIZES = [0, 1, 2, 63, 64, 65, 1000, 4095, 4096, 4097, 100_003, 1_000_000]


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("n", SIZES)
def test_sort_random(eng, kb, n):
    rng = np.random.default_rng(n + kb)
    for bits in sorted({8 * kb, 20, 13}):
        say(f"sort kb={kb} n={n} bits={bits}")
        a = rand_keys(rng, n, kb, bits)
        t = to_dev(a, kb)
        eng.sort_keys(t, bits)
        assert np.array_equal(to_host(t, kb), np.sort(a))


@pytest.mark.parametrize("kb", [4, 8])
def test_sort_special(eng, kb):
    n = 50_001
    top = np.iinfo(U[kb]).max
    cases = {
        "equal": np.full(n, 7, dtype=U[kb]),
        "sorted": np.arange(n, dtype=U[kb]),
        "reversed": np.arange(n, dtype=U[kb])[::-1].copy(),
        "extremes": np.array([top, 0, top, 1, 0, top - 1] * 1000, dtype=U[kb]),
        "two_values": np.where(np.arange(n) % 3 == 0, top, 0).astype(U[kb]),
    }
    for name, a in cases.items():
        say(f"sort special {name} kb={kb}")
        t = to_dev(a, kb)
        eng.sort_keys(t, 0)
        assert np.array_equal(to_host(t, kb), np.sort(a)), name


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("n,nf,span", [(0, 10, 100), (1, 0, 10), (5000, 0, 1000),
                                        (20_000, 30_000, 60_000), (100_000, 5_000, 1 << 30),
                                        (50_000, 2_000_000, 4_000_000), (300_000, 1000, 2000),
                                        (100_000, 1_500_000, 3_000_000),
                                        (9_000, 600_000, 10_000_000),
                                        # full no larger than the candidates (merge-path
                                        # tiles): overlapping, few long runs, nearly all
                                        # candidates present, full around the candidates
                                        (1_000_000, 900_000, 1_500_000), (2_000_000, 100, 50),
                                        (500_000, 400_000, 400_000), (70_001, 70_000, 1 << 40)])
def test_unique_diff(eng, kb, n, nf, span):
    import torch
    say(f"unique_diff kb={kb} n={n} nf={nf} span={span}")
    rng = np.random.default_rng(n * 7 + nf)
    c = np.sort(rng.integers(0, span, size=n).astype(U[kb]))
    f = np.unique(rng.integers(0, span, size=nf).astype(U[kb]))
    out, nu = eng.unique_diff(to_dev(c, kb), to_dev(f, kb) if len(f) else
                              torch.empty(0, dtype=getattr(torch, "int32" if kb == 4 else "int64"),
                                          device="cuda"))
    want = np.setdiff1d(np.unique(c), f)
    assert nu == len(np.unique(c))
    assert np.array_equal(to_host(out, kb), want)


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("na,nb", [(0, 0), (0, 5), (7, 0), (1, 1), (2048, 1), (3000, 5000),
                                   (1_000_000, 1234), (17, 400_000), (500_000, 500_000)])
def test_merge(eng, kb, na, nb):
    say(f"merge kb={kb} na={na} nb={nb}")
    rng = np.random.default_rng(na + 3 * nb)
    allk = np.unique(rand_keys(rng, 2 * (na + nb) + 10, kb, 8 * kb))
    rng.shuffle(allk)
    a = np.sort(allk[:na])
    b = np.sort(allk[na:na + nb])
    out = eng.merge(to_dev(a, kb), to_dev(b, kb))
    assert np.array_equal(to_host(out, kb), np.sort(np.concatenate([a, b])))


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("n", [0, 1, 1000, 100_000])
def test_hisa_query(eng, kb, n):
    import torch
    say(f"hisa kb={kb} n={n}")
    rng = np.random.default_rng(n + 11)
    shift = 16 if kb == 4 else 32
    jc_max = (1 << (32 - shift)) - 1 if kb == 4 else (1 << 32) - 1
    # skewed join keys: a few long runs and many short ones
    jc = np.concatenate([rng.integers(0, min(jc_max, 50_000) + 1, size=n),
                         np.full(n // 3, 5), np.full(n // 7, min(jc_max, 0xFFFFFFFF))])
    other = rng.integers(0, 1 << shift, size=len(jc))
    keys = np.unique((jc.astype(np.uint64) << np.uint64(shift)) | other.astype(np.uint64))
    keys = keys.astype(U[kb])
    jk = (keys.astype(np.uint64) >> np.uint64(shift)).astype(np.uint32)
    q = np.concatenate([np.unique(jk), rng.integers(0, min(jc_max, 60_000) + 1, size=2000),
                        np.array([0, 1, min(jc_max, 0xFFFFFFFF)])]).astype(np.uint32)
    tq = torch.from_numpy(q.view(np.int32)).cuda()
    st, ln, runs = eng.hisa_query(to_dev(keys, kb), shift, tq)
    lo = np.searchsorted(jk, q, side="left")
    hi = np.searchsorted(jk, q, side="right")
    want_len = (hi - lo).astype(np.int64)
    want_start = np.where(want_len > 0, lo, 0)
    assert runs == len(np.unique(jk))
    assert np.array_equal(ln.cpu().numpy().astype(np.int64), want_len)
    assert np.array_equal(st.cpu().numpy(), want_start)


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("n,dist", [(0, "uniform"), (1, "uniform"), (100, "uniform"),
                                    (100_000, "uniform"), (100_000, "clustered"),
                                    (1_000_000, "zipf")])
def test_learned_query(eng, kb, n, dist):
    import torch
    say(f"learned kb={kb} n={n} {dist}")
    key_bits = 32 if kb == 4 else 44
    top = (1 << key_bits) - 1
    rng = np.random.default_rng(n + kb)
    if dist == "uniform":
        raw = rng.integers(0, top + 1, size=n, dtype=np.uint64)
    elif dist == "clustered":
        centers = rng.integers(0, top + 1, size=20, dtype=np.uint64)
        raw = (centers[rng.integers(0, 20, size=n)] +
               rng.integers(0, 5000, size=n, dtype=np.uint64)) & np.uint64(top)
    else:
        raw = (rng.zipf(1.3, size=n).astype(np.uint64) * np.uint64(977)) & np.uint64(top)
    keys = np.unique(raw).astype(U[kb])
    q = np.concatenate([keys, keys + 1, rng.integers(0, top + 1, size=5000, dtype=np.uint64),
                        np.array([0, top, top - 1], dtype=np.uint64)]).astype(np.uint64)
    q = (q & np.uint64(top)).astype(U[kb])
    pos = eng.learned_query(to_dev(keys, kb), key_bits, to_dev(q, kb))
    want = np.searchsorted(keys, q, side="left")
    assert np.array_equal(pos.cpu().numpy().astype(np.int64), want)


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("reps,nf,span", [(4, 2_000_000, 4_000_000), (3, 3_000_000, 1 << 31),
                                           (1, 5_000_000, 6_000_000)])
def test_unique_diff_repeats_far_apart(eng, kb, reps, nf, span):
    """Candidates far apart in a large full (tiles whose slice of full is
    searched through the sampled index, not streamed), each repeated: only
    the first of a run is tested and kept; the result is the set definition's."""
    rng = np.random.default_rng(reps * 11 + nf)
    f = np.unique(rng.integers(0, span, size=nf).astype(np.uint64)).astype(U[kb])
    d = np.unique(rng.integers(0, span, size=30_000).astype(np.uint64))
    # half of the distinct candidates are members of full
    d = np.unique(np.concatenate([d[: len(d) // 2], rng.choice(f.astype(np.uint64), 15_000)]))
    c = np.sort(np.repeat(d.astype(U[kb]), reps))
    out, nu = eng.unique_diff(to_dev(c, kb), to_dev(f, kb))
    assert nu == len(d)
    assert np.array_equal(to_host(out, kb), np.setdiff1d(d.astype(U[kb]), f))
