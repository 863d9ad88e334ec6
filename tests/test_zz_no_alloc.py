"""sim_loss_noalloc (the loss entry point that allocates nothing, its
per-window partials in the library's static device scratch) against
sim_loss on the same inputs: identical loss and gradient, bit for bit (the
same kernels in the same order), on two calls in a row, the second with a
smaller batch, and the batch limit refused on the host."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_loss_noalloc_equals_loss(torch):
    import paper_2105_05821_amd as sn
    layers = synth.net_c3_hybrid()
    ws, bs = synth.init_weights(9, layers, out_bias=None, out_gain=1.0)
    pred = sn.Predictor(layers, sn.SIM_FP32)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    gen = torch.Generator(device="cpu").manual_seed(3)
    for B in (3000, 517):
        z = (4 * torch.randn((B, 802), generator=gen)).cuda()
        lat = torch.randint(0, 450, (B, 2), generator=gen, dtype=torch.int32).cuda()
        l1, d1 = pred.loss(z, lat)
        # poisoned outputs: every element must be written
        out = (torch.full((), float("nan"), device="cuda"),
               torch.full((B, 802), float("nan"), device="cuda"))
        l2, d2 = pred.loss(z, lat, out=out, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(l1, l2), (B, float(l1), float(l2))
        assert torch.equal(d1, d2), B
        assert np.isfinite(float(l2))
    z = torch.zeros((sn.NOALLOC_MAX_B + 1, 802), device="cuda")
    lat = torch.zeros((z.shape[0], 2), dtype=torch.int32, device="cuda")
    with pytest.raises(sn.SimError, match="SIM_EINVAL"):
        pred.loss(z, lat, noalloc=True)
    pred.close()
