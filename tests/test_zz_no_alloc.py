"""The allocation-free matching entry point (pg_match_descriptors_noalloc,
scratch in the library's fixed device array) against the allocating one
(pg_match_descriptors), through the C ABI: bit-equal matches and distances on
two calls in a row, the second smaller than the first (the array keeps the
first call's contents), and a call larger than the array refused before any
work is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def unit(rng, n, dim):
    x = rng.normal(size=(n, dim))
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


def both(sets, pairs, ratio):
    import torch
    from paper_2108_00516_amd import frontend
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)
    desc = torch.from_numpy(np.ascontiguousarray(np.concatenate(sets, axis=0))).cuda()
    ref = frontend.match_descriptors(desc, off, pairs, ratio)
    got = frontend.match_descriptors(desc, off, pairs, ratio, noalloc=True)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got]


def test_noalloc_equals_allocating_entry_point():
    rng = np.random.default_rng(5)
    print("no-alloc matching: 8 sets x 500 x 128, 28 pairs, then 3 sets, 3 pairs", flush=True)
    sets = [unit(rng, 500, 128) for _ in range(8)]
    for s in sets[1:]:
        s[:200] = sets[0][:200] + rng.normal(scale=0.01, size=(200, 128)).astype(np.float32)
    pairs = [(i, j) for i in range(8) for j in range(i + 1, 8)]
    ref, got = both(sets, pairs, 0.9)
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
    assert (ref[0] >= 0).sum() > 1000
    # a second, smaller call: the array still holds the first call's records
    small = [unit(rng, n, 128) for n in (70, 33, 129)]
    small[1][:20] = small[0][:20]
    ref, got = both(small, [(0, 1), (2, 0), (1, 2)], 1.0)
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)


def test_noalloc_refuses_calls_beyond_its_scratch():
    import torch
    from paper_2108_00516_amd import frontend
    desc = torch.zeros((4096, 32), dtype=torch.float32, device="cuda")
    # 3 pairs x 64 row tiles x 4096 columns > 2^19 partial records
    with pytest.raises(frontend.FrontendError, match="CAPACITY"):
        frontend.match_descriptors(desc, [0, 4096], [(0, 0)] * 3, noalloc=True)
    m, _, _ = frontend.match_descriptors(desc[:64].contiguous(), [0, 64], [(0, 0)], noalloc=True)
    torch.cuda.synchronize()
    assert m.shape[0] == 64
