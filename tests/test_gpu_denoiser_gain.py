"""What the trained denoiser gains over the method without it: the transport
generates low/high-history dose pairs on small synthetic CTs, the network is
trained on the GPU by the library's own forward/backward/Adam kernels, and
on held-out cases its output is closer to the high-history reference than
the noisy input it was given (mean relative error over the dose region)."""
import sys

import numpy as np
import pytest

from paper_1409_8336_amd import denoise, pmc, synth, unet

pytestmark = pytest.mark.gpu

SHAPE = (80, 64, 64)          # z, y, x voxels of 2 mm
N_TRAIN, N_TEST = 24, 4
N_LOW, N_HIGH = 20_000, 2_000_000


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(i):
    rng = np.random.default_rng(5000 + i)
    nz, ny, nx = SHAPE
    hu = synth.ct_phantom(nx, ny, nz, 0.2, seed=5000 + i, counts=(1, 1, 1), ti_depth_cm=None)
    spots = synth.training_field(rng, (0.1 * nx, 0.1 * ny), e_lo=70.0, e_hi=130.0)
    return hu, spots


def _mre(a, ref):
    m = ref >= 0.1 * ref.max()
    return float(np.mean(np.abs(a[m] - ref[m]) / ref[m]))


def test_trained_denoiser_beats_its_noisy_input():
    import torch
    _say("case: denoiser training gain")
    e = pmc.Engine(0)
    e.load_physics(synth.nuclear_data())
    mt = synth.material_table()
    n = N_TRAIN + N_TEST
    low = torch.empty((n,) + SHAPE, dtype=torch.float32, device="cuda")
    high = torch.empty_like(low)
    rho = torch.empty_like(low)
    d = torch.empty(SHAPE, dtype=torch.float64, device="cuda")
    for i in range(n):
        hu, spots = _case(i)
        e.load_geometry(hu, (0.2, 0.2, 0.2), mt)
        pmc.pmc_geometry_density(e.ctx, 0, rho[i])
        e.run_spots_dev(spots, N_LOW, 100 + i, d)
        low[i].copy_(d)
        e.run_spots_dev(spots, N_HIGH, 200 + i, d)
        high[i].copy_(d)
    torch.cuda.synchronize()
    e.close()
    net = unet.UNet((1,) + SHAPE, seed=3)
    # the library's training recipe (cosine decay, gradient-norm clipping) for
    # a fixed number of updates of two volumes each, at most 45 s: a constant
    # learning rate without clipping can spike and leave Adam frozen
    hist = denoise.train(net, {"low": low, "rho": rho, "high": high}, list(range(N_TRAIN)), 45.0,
                         lr_max=1e-3, lr_min=1e-5, seed=0, max_steps=10_000, batch=2, clip=3.0,
                         log=lambda *a: None)
    torch.cuda.synchronize()
    losses = [h[2] for h in hist]
    _say("trained %d steps (%d clipped), loss first 50 %.3e last 50 %.3e"
         % (len(hist), net.n_clipped, np.mean(losses[:50]), np.mean(losses[-50:])))
    out = torch.empty(SHAPE, dtype=torch.float32, device="cuda")
    gains = []
    for i in range(N_TRAIN, n):
        net.forward(low[i], rho[i], out)
        torch.cuda.synchronize()
        ref = high[i].cpu().numpy().astype(np.float64)
        m_low = _mre(low[i].cpu().numpy().astype(np.float64), ref)
        m_den = _mre(out.cpu().numpy().astype(np.float64), ref)
        gains.append(m_low / m_den)
        _say("held-out %d: MRE noisy %.4f denoised %.4f" % (i, m_low, m_den))
    net.close()
    assert np.mean(losses[-50:]) < np.mean(losses[:50])
    # every held-out case improves, and on average by at least a quarter
    assert min(gains) > 1.0 and np.mean(gains) > 1.25, gains
