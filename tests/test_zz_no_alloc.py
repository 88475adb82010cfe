"""The data gradient that allocates nothing (pmc_nn_conv3d_backward_data_noalloc,
include/pmc_unet.h) against the allocating entry point, through the C ABI:
the same kernels on the same BF16 inputs, so the outputs must be equal bit
for bit, on two calls in a row (the second smaller, over the workspace the
first one left behind), plus the oracle's bound on the second call and the
workspace limit's rejection on the host.
"""
import sys

import numpy as np
import pytest

from oracle import denoiser_oracle as D
from paper_1409_8336_amd import pmc, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda()


def test_noalloc_data_gradient_equals_the_allocating_one():
    import torch
    from paper_1409_8336_amd import unet as U
    # the larger layer first (fills more of the workspace), then a smaller one
    for cin, cout, shape in ((192, 64, (1, 3, 4, 68)), (16, 32, (2, 3, 4, 40))):
        _say("case: no-alloc data gradient cin=%d cout=%d shape=%s" % (cin, cout, shape))
        rng = np.random.default_rng(cin * 7 + cout)
        gb, g = synth.bf16_normal(rng, shape + (cout,))
        wb, w = synth.conv_weights(rng, cin, cout)
        dx_ref = torch.zeros(shape + (cin,), dtype=torch.int16, device="cuda")
        dx_new = torch.full(shape + (cin,), 0x7FC0, dtype=torch.int16, device="cuda")   # NaN pattern
        U.pmc_nn_conv3d_backward_data(_dev(gb), _dev(wb), dx_ref)
        U.pmc_nn_conv3d_backward_data_noalloc(_dev(gb), _dev(wb), dx_new)
        torch.cuda.synchronize()
        a, b = dx_ref.cpu().numpy(), dx_new.cpu().numpy()
        assert np.array_equal(a, b), int((a != b).sum())
        # and the oracle's bound (BF16 output rounding, FP32 sums of 27 cout terms)
        o = D.conv3d_backward_data(g, w, cin)
        s = D.conv3d_backward_data(np.abs(g), np.abs(w), cin)
        r = synth.bf16_values(b.view(np.uint16))
        bound = 2.0 ** -8 * np.abs(o) + 2.0 * (27 * cout + 1) * 2.0 ** -24 * s + 1e-30
        assert not (np.abs(r - o) > bound).any()


def test_noalloc_data_gradient_rejects_a_workspace_too_large():
    """cin * round_up(27 cout, 32) above 2^20 entries is refused before any
    device work (256 x 6912 = 1,769,472)."""
    import torch
    from paper_1409_8336_amd import unet as U
    dy = torch.zeros((1, 1, 1, 8, 256), dtype=torch.int16, device="cuda")
    w = torch.zeros((256, 27 * 256), dtype=torch.int16, device="cuda")
    dx = torch.zeros((1, 1, 1, 8, 256), dtype=torch.int16, device="cuda")
    with pytest.raises(pmc.PMCError) as ei:
        U.pmc_nn_conv3d_backward_data_noalloc(dy, w, dx)
    assert ei.value.status == pmc.PMC_ERR_RANGE
