"""hb_mlp_forward_noalloc (hidden activations in the library's fixed device
array) against hb_mlp_forward (the handle's own buffers), through the C ABI:
two calls in a row, the second with a smaller batch, and the size limit.
Both run the same kernels in the same order, so the outputs are identical."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2411_14315_amd as hbl  # noqa: E402
from paper_2411_14315_amd.learned import MLP  # noqa: E402

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward():
    net = MLP([23, 256, 256, 64], seed=7)
    rng = np.random.default_rng(3)
    for B in (512, 37):
        X = torch.from_numpy(rng.normal(size=(B, 23)).astype(np.float32)).cuda()
        ref = net.forward(X)
        Y = torch.full((B, 64), np.nan, dtype=torch.float32, device="cuda")
        net.forward_noalloc(X, Y)
        torch.cuda.synchronize()
        print("B", B, "max |diff|", float((Y - ref).abs().max()), flush=True)
        assert torch.equal(Y, ref)
    # a wider network and a batch at the limit of the 16 MiB array
    wide = MLP([5, 1024, 64], seed=1)
    B = (1 << 20) // 1024
    X = torch.from_numpy(rng.normal(size=(B, 5)).astype(np.float32)).cuda()
    Y = torch.empty((B, 64), dtype=torch.float32, device="cuda")
    wide.forward_noalloc(X, Y)
    assert torch.equal(Y, wide.forward(X))
    X2 = torch.zeros((B + 1, 5), dtype=torch.float32, device="cuda")
    Y2 = torch.empty((B + 1, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(hbl.HBError) as e:
        wide.forward_noalloc(X2, Y2)
    assert e.value.status == hbl.HB_ERR_ARG and "scratch" in str(e.value)
    net.close()
    wide.close()
