"""Run-to-run determinism of the GPU path (through the C ABI).

The kernels combine partial results only with commutative atomics (or, add,
min, max) and every list is written in a canonical grouping, so two runs of the
same call give identical core numbers and identical result fields, whatever
the order in which the blocks ran.  Checked on a power-law graph with hubs
(split into slices), exact and sampled, with Alg. 7's densest core."""
import sys

import numpy as np
import pytest

import graphgen as gg

torch = pytest.importorskip("torch")
kh = pytest.importorskip("paper_2112_06154_amd")

pytestmark = pytest.mark.gpu

FIELDS = ("M_used", "M_dense_used", "rounds", "max_core", "dense_k", "dense_size", "dense_density")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("h,eps", [(2, 0.0), (3, 0.0), (2, 0.5), (3, 0.5)])
def test_two_runs_are_identical(ctx, h, eps):
    g = gg.chung_lu(60000, 600000, 2.1, seed=4)
    G = kh.Graph.from_gg(ctx, g)
    print("determinism", h, eps, flush=True)
    sys.stdout.flush()
    runs = [kh.core(G, h, epsilon=eps, seed=9, dense=True, prune=True) for _ in range(2)]
    (c0, r0), (c1, r1) = runs
    assert c0.tobytes() == c1.tobytes()
    for k in FIELDS:
        assert r0[k] == r1[k], k
