"""Host-side sizing of the sampled peel's hub slices (no GPU).

The library sizes the slice buffers once per run from nnz and the slice size S
(2 nnz / S + 1 partial-list slots, nnz / 1025 + 1 + slots work items,
nnz / S + 1 split hubs) and cuts each hub of degree d > 1024 into
ceil(d / s) slices of s = max(S, ceil(d / 256)) arcs when that is more than
one.  These checks run the same arithmetic over many degree sequences and
confirm that no worklist of hubs can need more than the sized buffers."""
import numpy as np
import pytest

HUB_DEGREE = 1024
MERGE_THREADS = 256


def slices(deg, S):
    sl = max(S, -(-deg // MERGE_THREADS))
    return -(-deg // sl)


@pytest.mark.parametrize("S", [1, 7, 64, 128, 300, 1024, 8192, 100_000])
@pytest.mark.parametrize("seed", range(6))
def test_slice_buffers_hold_every_worklist(S, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 5000))
    # power-law-ish degrees with a few very large hubs
    deg = np.minimum((rng.pareto(1.1, n) * 20).astype(np.int64) + 1, 3_000_000)
    nnz = int(deg.sum())
    slots_cap = 2 * (nnz // S) + 1
    units_cap = nnz // (HUB_DEGREE + 1) + 1 + slots_cap
    giants_cap = nnz // S + 1
    hubs = deg[deg > HUB_DEGREE]            # the worst case: every hub in one worklist
    ns = np.array([slices(int(d), S) for d in hubs], dtype=np.int64)
    split = ns > 1
    assert int(ns[split].sum()) <= slots_cap
    assert int(ns[split].sum()) + int((~split).sum()) <= units_cap
    assert int(split.sum()) <= giants_cap
    assert (ns <= MERGE_THREADS).all()
    # every slice covers its share of the arcs exactly once
    for d in hubs[:50]:
        d = int(d)
        k = slices(d, S)
        sl = max(S, -(-d // MERGE_THREADS))
        ranges = [(j * sl, min(d, (j + 1) * sl)) for j in range(k)]
        assert ranges[0][0] == 0 and ranges[-1][1] == d
        assert all(a < b for a, b in ranges)
