"""The entry point that allocates nothing (hl_sort_keys_noalloc) against the
allocating one (hl_sort_keys), through the C ABI: bit-exact on two calls in
a row, the second smaller than the first, for 32- and 64-bit keys (with a
digit count that leaves the result in the scratch copy and one that does
not), plus its size limit and the argument checks it shares."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def engine():
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    return pkg.Engine(device=0, stream=torch.cuda.current_stream())


def keys(n, key_bytes, bits, seed):
    import torch
    rng = np.random.default_rng(seed)
    if key_bytes == 4:
        v = rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(np.uint32)
        return torch.from_numpy(v.view(np.int32)).cuda()
    v = rng.integers(0, 1 << min(bits, 63), size=n, dtype=np.uint64)
    if bits == 64:
        v |= rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63)
    return torch.from_numpy(v.view(np.int64)).cuda()


@pytest.mark.parametrize("key_bytes,bits,sizes", [
    (4, 32, (12_000_000, 100_003)),
    (4, 20, (3_000_001, 4_097)),
    (8, 44, (7_000_000, 333_333)),
    (8, 64, (2_000_000, 65_537)),
])
def test_noalloc_sort_equals_allocating_sort(key_bytes, bits, sizes):
    e = engine()
    try:
        for i, n in enumerate(sizes):
            src = keys(n, key_bytes, bits, seed=100 * key_bytes + bits + i)
            a = src.clone()
            b = src.clone()
            e.sort_keys(a, bits)
            e.sort_keys_noalloc(b, bits)
            assert bool((a == b).all()), f"call {i} ({n} keys) differs"
            # and both are the sorted input (unsigned order)
            want = np.sort(src.cpu().numpy().view(np.uint32 if key_bytes == 4 else np.uint64))
            got = b.cpu().numpy().view(want.dtype)
            assert np.array_equal(got, want)
    finally:
        e.close()


def test_noalloc_limits_and_errors():
    import torch
    import paper_2311_02206_amd as pkg
    e = engine()
    try:
        limit = pkg.hisalog.NOALLOC_SCRATCH_BYTES
        too_many = limit // 4 + 1  # 4-byte keys alone would fill the scratch
        big = torch.zeros(too_many, dtype=torch.int32, device="cuda")
        with pytest.raises(pkg.HlError) as ei:
            e.sort_keys_noalloc(big, 32)
        assert ei.value.code == pkg.hisalog.HL_E_CAPACITY
        del big
        # a failed call leaves the engine usable, and 0 or 1 keys are a no-op
        one = torch.tensor([7], dtype=torch.int64, device="cuda")
        e.sort_keys_noalloc(one, 64)
        assert one.item() == 7
        empty = torch.empty(0, dtype=torch.int32, device="cuda")
        e.sort_keys_noalloc(empty, 32)
        with pytest.raises(pkg.HlError) as ei:
            e.sort_keys_noalloc(torch.zeros(10, dtype=torch.int32, device="cuda"), 40)
        assert ei.value.code == pkg.hisalog.HL_E_INVALID
        x = keys(1000, 4, 32, seed=5)
        y = x.clone()
        e.sort_keys_noalloc(x, 32)
        e.sort_keys(y, 32)
        assert bool((x == y).all())
    finally:
        e.close()
