"""knng_leaf_search_noalloc (scratch from the library's fixed device array,
no allocation) against knng_leaf_search on the same inputs, through the C
ABI: identical ids and distances, on two calls in a row, the second with a
smaller input (the array keeps the first call's contents)."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1701_08475_amd import knng
    knng.lib()
    return knng


def _leaves(orc, X, T, L, ml, seed):
    import torch
    perms, offs = [], []
    for t in range(T):
        tr = orc.tree(X, L, ml, 10, seed, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    return (torch.from_numpy(np.stack(perms)).cuda(),
            [torch.from_numpy(o).cuda() for o in offs])


@pytest.mark.parametrize("first,second", [
    # (n, D, k, trees, leaf_max, precision): leaves above 128 points take the
    # size buckets of the reduced path; one tree writes the output directly
    ((6000, 32, 10, 3, 200, "fp8"), (2500, 24, 8, 2, 60, "fp32")),
    ((5000, 40, 12, 2, 150, "fp16"), (3000, 40, 12, 1, 150, "bf16")),
])
def test_noalloc_equals_leaf_search(K, orc, first, second):
    import torch
    for call, (n, D, k, T, L, prec) in enumerate((first, second)):
        X = datagen.random_points(n, D, 31 + call, "normal")
        Xd = to_dev(X)
        perms, offs = _leaves(orc, X, T, L, k + 1, 7 + call)
        log("noalloc call %d: n=%d D=%d k=%d T=%d L=%d %s" % (call, n, D, k, T, L, prec))
        a_ids, a_d = K.leaf_search(Xd, k, perms, offs, precision=prec)
        b_ids, b_d = K.leaf_search(Xd, k, perms, offs, precision=prec, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(a_ids, b_ids)
        assert torch.equal(a_d.view(torch.int32), b_d.view(torch.int32))


def test_noalloc_rejects_what_does_not_fit(K):
    import torch
    n, T, k = 300_000, 8, 32
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    perms = torch.arange(n, dtype=torch.int32, device="cuda").repeat(T, 1)
    offs = [torch.tensor([0, n // 2, n], dtype=torch.int32, device="cuda")] * T
    with pytest.raises(K.KnngError) as e:
        K.leaf_search(X, k, perms, offs, noalloc=True)
    assert e.value.status == K.KNNG_ERR_UNSUPPORTED
