"""Seeded generators: determinism (digests pinned), distinctness, shapes."""

import hashlib

import numpy as np

import workloads as w


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def test_digests_are_stable():
    assert digest(w.erdos_renyi(1000, 3000, 0xC1)) == "950f1155aafd5749"
    assert digest(w.rmat(10, 3000, 5)) == "5cd365a159f387cd"
    assert digest(w.random_tree(5000, 0xC2B)) == "d00fd2aaaeffb276"
    assert digest(w.zipf_pairs(1 << 12, 2000, 1.2, 0xC3, 0)) == "ea86097b9e5ec55c"
    c = w.cspa()["edb"]
    assert c["Assign"].shape == (6250, 2) and c["Dereference"].shape == (2343, 2)
    assert digest(np.concatenate([c["Assign"], c["Dereference"]])) == "c1c00eaab811b86c"
    n, e = w.batched_reach_instances(8, 0xC4)
    assert n.tolist() == [84, 601, 1197, 2158, 162, 2772, 95, 85]
    assert digest(np.concatenate(e)) == "b384fb22bfa55c90"


def distinct_no_self(e):
    key = (e[:, 0].astype(np.uint64) << np.uint64(32)) | e[:, 1]
    return len(np.unique(key)) == len(e) and not np.any(e[:, 0] == e[:, 1])


def test_er_shape():
    e = w.erdos_renyi(1000, 3000, 0xC1)
    assert e.shape == (3000, 2) and e.dtype == np.uint32
    assert distinct_no_self(e) and e.max() < 1000


def test_rmat_shape_and_skew():
    e = w.rmat(12, 20000, 1)
    assert e.shape == (20000, 2) and distinct_no_self(e) and e.max() < 4096
    # quadrant (0,0) is the heaviest: low ids dominate the sources
    assert np.mean(e[:, 0] < 2048) > 0.7


def test_tree_shape():
    e = w.random_tree(5000, 3)
    assert e.shape == (4999, 2)
    assert np.array_equal(e[:, 1], np.arange(1, 5000))
    assert np.all(e[:, 0] < e[:, 1])
    _, c = np.unique(e[:, 0], return_counts=True)
    assert c.min() >= 1 and c.max() <= 4


def test_zipf_orientations():
    lit = w.zipf_pairs(1 << 14, 5000, 1.2, 9, 0, orient="literal")
    rnk = w.zipf_pairs(1 << 14, 5000, 1.2, 9, 0, orient="by_rank")
    src = w.zipf_pairs(1 << 14, 5000, 1.2, 9, 0, orient="src_zipf")
    for e in (lit, rnk, src):
        assert e.shape == (5000, 2) and distinct_no_self(e)
    assert np.all(rnk[:, 0] < rnk[:, 1])
    # id 0 (rank 1) is a hub
    assert np.mean(lit[:, 0] == 0) > 0.05


def test_batched_instances():
    n, e = w.batched_reach_instances(64, 0xC4)
    assert len(e) == 64 and n.min() >= 32 and n.max() <= 4096
    for k in range(64):
        m = len(e[k])
        assert 2 * n[k] <= m + 1 and m <= 4 * n[k]
        assert distinct_no_self(e[k]) and e[k].max() < n[k]
