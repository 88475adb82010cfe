"""Denoiser kernels and the gamma index on the GPU against the FP64 oracle,
called through the C ABI (include/pmc_unet.h).

Tolerances (derived from the arithmetic):
* inputs and weights are bfloat16 values, exact in FP64 on the oracle side;
  the kernels sum K products in FP32 (any order, every addition rounded at
  most once, truncation allowed: at most 2*K*2^-24 * S, S = the same sum over
  absolute values) and, for bfloat16 outputs, round once to nearest
  (unit roundoff 2^-8: 8 significant bits).  Bound:
  |gpu - oracle| <= 2^-8 |oracle| + 2 (K + 1) 2^-24 S.
* whole network: every one of the 7 convolutions rounds its weights and its
  output to bfloat16 (2^-8 each) in the forward pass and its gradients again
  in the backward pass; about 2 x 14 such roundings compound to well under
  2^-5 relative (L2) in the outputs and per-layer gradients.
* gamma: evaluated in FP64 with FP32 search offsets (relative 2^-23), output
  FP32: 1e-5 relative.  The pass decision is compared where the oracle's
  gamma is not within 1e-4 of 1.
"""
import sys

import numpy as np
import pytest

from oracle import denoiser_oracle as D
from paper_1409_8336_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda()


def _host_bf16(t):
    return synth.bf16_values(t.cpu().numpy().view(np.uint16))


def _unet():
    from paper_1409_8336_amd import unet
    return unet


def _conv_bound(o, s, k):
    return 2.0 ** -8 * np.abs(o) + 2.0 * (k + 1) * 2.0 ** -24 * s + 1e-30


CONV_CASES = [
    # (cin, cout, (n, d, h, w))
    (8, 16, (1, 4, 5, 70)),
    (16, 32, (2, 3, 4, 66)),
    (24, 24, (1, 5, 3, 40)),
    (64, 128, (1, 3, 3, 72)),
    (192, 64, (1, 2, 3, 68)),
    (48, 16, (1, 4, 4, 130)),
]


@pytest.mark.parametrize("cin,cout,shape", CONV_CASES)
def test_conv_forward(cin, cout, shape):
    import torch
    _say("case: conv forward cin=%d cout=%d shape=%s" % (cin, cout, shape))
    U = _unet()
    rng = np.random.default_rng(cin * 1000 + cout)
    xb, x = synth.bf16_normal(rng, shape + (cin,))
    wb, w = synth.conv_weights(rng, cin, cout)
    b = rng.normal(0, 0.1, cout).astype(np.float32)
    y = torch.zeros(shape + (cout,), dtype=torch.int16, device="cuda")
    for relu in (False, True):
        U.pmc_nn_conv3d_forward(_dev(xb), _dev(wb), torch.from_numpy(b).cuda(), y, relu=relu)
        torch.cuda.synchronize()
        o = D.conv3d(x, w, b, relu=relu)
        s = D.conv3d(np.abs(x), np.abs(w), np.abs(b))
        g = _host_bf16(y)
        bound = _conv_bound(o, s, 27 * cin)
        bad = np.abs(g - o) > bound
        assert not bad.any(), (relu, int(bad.sum()), float(np.abs(g - o).max()))


@pytest.mark.parametrize("cin,cout,shape", CONV_CASES)
def test_conv_backward_data(cin, cout, shape):
    import torch
    _say("case: conv backward data cin=%d cout=%d shape=%s" % (cin, cout, shape))
    U = _unet()
    rng = np.random.default_rng(cin * 1000 + cout + 1)
    gb, g = synth.bf16_normal(rng, shape + (cout,))
    wb, w = synth.conv_weights(rng, cin, cout)
    dx = torch.zeros(shape + (cin,), dtype=torch.int16, device="cuda")
    U.pmc_nn_conv3d_backward_data(_dev(gb), _dev(wb), dx)
    torch.cuda.synchronize()
    o = D.conv3d_backward_data(g, w, cin)
    s = D.conv3d_backward_data(np.abs(g), np.abs(w), cin)
    r = _host_bf16(dx)
    bad = np.abs(r - o) > _conv_bound(o, s, 27 * cout)
    assert not bad.any(), (int(bad.sum()), float(np.abs(r - o).max()))


@pytest.mark.parametrize("cin,cout,shape", CONV_CASES)
def test_conv_backward_weight(cin, cout, shape):
    """dw += sum over voxels; dw starts from a nonzero value to check the
    accumulation."""
    import torch
    _say("case: conv backward weight cin=%d cout=%d shape=%s" % (cin, cout, shape))
    U = _unet()
    rng = np.random.default_rng(cin * 1000 + cout + 2)
    xb, x = synth.bf16_normal(rng, shape + (cin,))
    gb, g = synth.bf16_normal(rng, shape + (cout,))
    k = D.kp(cin)
    dw0 = rng.normal(0, 1.0, (cout, k)).astype(np.float32)
    dw0[:, 27 * cin:] = 0.0
    dw = torch.from_numpy(dw0.copy()).cuda()
    U.pmc_nn_conv3d_backward_weight(_dev(xb), _dev(gb), dw)
    torch.cuda.synchronize()
    o = dw0.astype(np.float64) + D.conv3d_backward_weight(x, g, k)
    s = np.abs(dw0) + D.conv3d_backward_weight(np.abs(x), np.abs(g), k)
    r = dw.cpu().numpy().astype(np.float64)
    nvox = int(np.prod(shape))
    bad = np.abs(r - o) > 2.0 * (nvox + 1) * 2.0 ** -24 * s + 1e-30
    assert not bad.any(), (int(bad.sum()), float(np.abs(r - o).max()))
    assert np.all(r[:, 27 * cin:] == 0.0)


@pytest.mark.parametrize("cin,cout,level", [(8, 16, 0), (48, 16, 0), (192, 64, 2)])
def test_conv_forward_full_size_sampled(cin, cout, level):
    """At the full 160x128x128 input (level 0) or its level-2 grid, 300
    sampled output voxels (corners, faces and random interior) against the
    oracle's one-voxel-at-a-time sum."""
    import torch
    shape = (1, 160 >> level, 128 >> level, 128 >> level)
    _say("case: conv forward full size cin=%d cout=%d shape=%s" % (cin, cout, shape))
    U = _unet()
    rng = np.random.default_rng(77 + cin)
    xb, x = synth.bf16_normal(rng, shape + (cin,))
    wb, w = synth.conv_weights(rng, cin, cout)
    b = rng.normal(0, 0.1, cout).astype(np.float32)
    y = torch.zeros(shape + (cout,), dtype=torch.int16, device="cuda")
    U.pmc_nn_conv3d_forward(_dev(xb), _dev(wb), torch.from_numpy(b).cuda(), y, relu=True)
    torch.cuda.synchronize()
    _, d, h, wd = shape
    pts = [(0, z, yy, xx) for z in (0, d - 1) for yy in (0, h - 1) for xx in (0, wd - 1)]
    pts += [(0, int(rng.integers(d)), int(rng.integers(h)), int(rng.integers(wd))) for _ in range(292)]
    o = D.conv3d_at(x, w, b, pts, relu=True)
    s = D.conv3d_at(np.abs(x), np.abs(w), np.abs(b), pts)
    yh = y.cpu().numpy().view(np.uint16)
    g = np.array([synth.bf16_values(yh[p]) for p in pts])
    bad = np.abs(g - o) > _conv_bound(o, s, 27 * cin)
    assert not bad.any(), (int(bad.sum()), float(np.abs(g - o).max()))


# ------------------------------------------------------------ network

def _net_inputs(rng, shape):
    dose = (rng.gamma(2.0, 1.0, shape) * 1e-3).astype(np.float32)
    rho = rng.uniform(0.2, 2.0, shape).astype(np.float32)
    target = (dose * rng.uniform(0.8, 1.2, shape)).astype(np.float32)
    return dose, rho, target


def _net_params(u, seed):
    """The library's initial parameters with nonzero biases and head, so
    that every gradient path is exercised; rounded to float32."""
    U = _unet()
    p = U.pmc_unet_get_params(u).astype(np.float64)
    rng = np.random.default_rng(seed)
    layout, ohw, ohb, n = D.param_layout()
    for name, ow, ob, cin, cout, k in layout:
        p[ob:ob + cout] = rng.normal(0, 0.05, cout)
    p[ohw:ohw + 16] = rng.normal(0, 0.1, 16)
    p[ohb] = 0.01
    return p.astype(np.float32)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape", [(1, 16, 16, 80), (2, 8, 16, 24)])
def test_network_forward_backward(shape):
    import torch
    _say("case: network forward/backward shape=%s" % (shape,))
    U = _unet()
    rng = np.random.default_rng(sum(shape))
    net = U.UNet(shape, seed=5)
    p = _net_params(net.u, 6)
    net.set_params(p)
    dose, rho, target = _net_inputs(rng, shape)
    td, tr, tt = (torch.from_numpy(a).cuda() for a in (dose, rho, target))
    out = torch.zeros_like(td)
    net.forward(td, tr, out)
    torch.cuda.synchronize()
    orc = D.UNetOracle(p.astype(np.float64))
    loss_o, grad_o, out_o = orc.loss_and_grad(dose.astype(np.float64), rho, target)
    scale = float(dose.max())
    head_g = (out.cpu().numpy() - dose) / scale
    head_o = (out_o - dose) / scale
    e_out = _rel_l2(head_g, head_o)
    net.zero_grads()
    loss_g = net.backward(td, tr, tt)
    grad_g = net.grads().astype(np.float64)
    _say("head rel-L2 %.2e loss gpu %.6e oracle %.6e" % (e_out, loss_g, loss_o))
    assert e_out <= 2.0 ** -5
    assert abs(loss_g - loss_o) <= 2.0 ** -5 * loss_o
    layout, ohw, ohb, n = D.param_layout()
    for name, ow, ob, cin, cout, k in layout:
        ew = _rel_l2(grad_g[ow:ow + cout * k], grad_o[ow:ow + cout * k])
        eb = _rel_l2(grad_g[ob:ob + cout], grad_o[ob:ob + cout])
        _say("%s dW rel-L2 %.2e db rel-L2 %.2e" % (name, ew, eb))
        assert ew <= 2.0 ** -5 and eb <= 2.0 ** -5, name
        # padding columns (and enc1's unused input channels) get no gradient
        gw = grad_g[ow:ow + cout * k].reshape(cout, k)
        assert np.all(gw[:, 27 * cin:] == 0.0)
    eh = _rel_l2(grad_g[ohw:ohb + 1], grad_o[ohw:ohb + 1])
    _say("head grad rel-L2 %.2e" % eh)
    assert eh <= 2.0 ** -5
    net.close()


def test_adam_step_and_bf16_refresh():
    """One Adam step against the oracle's Adam on the same (GPU) gradients,
    and the forward after the step equals the forward of a fresh network
    given the stepped parameters (the BF16 copies are refreshed)."""
    import torch
    _say("case: adam step")
    U = _unet()
    shape = (1, 8, 8, 16)
    rng = np.random.default_rng(31)
    net = U.UNet(shape, seed=3)
    p0 = _net_params(net.u, 4)
    net.set_params(p0)
    dose, rho, target = _net_inputs(rng, shape)
    td, tr, tt = (torch.from_numpy(a).cuda() for a in (dose, rho, target))
    net.backward(td, tr, tt)
    g = net.grads().astype(np.float64)
    lr = 1e-3
    net.adam_step(lr)
    torch.cuda.synchronize()
    p1 = net.params().astype(np.float64)
    orc = D.UNetOracle(p0.astype(np.float64))
    orc.adam_step(g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    dev = np.abs(p1 - orc.params)
    assert np.all(dev <= 1e-5 * lr + 2.0 ** -23 * np.abs(orc.params)), float(dev.max())
    assert np.all(net.grads() == 0.0)
    out1 = torch.zeros_like(td)
    net.forward(td, tr, out1)
    fresh = U.UNet(shape, seed=99)
    fresh.set_params(p1.astype(np.float32))
    out2 = torch.zeros_like(td)
    fresh.forward(td, tr, out2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    net.close()
    fresh.close()


def test_forward_region_equals_zero_padded_forward():
    """A grid smaller than the network's shape (the sides of a plan's CT need
    not divide by 8) gives, voxel for voxel, the output of the full-shape
    forward on the same grid zero-padded to the network's shape."""
    import torch
    _say("case: forward on a sub-grid")
    U = _unet()
    shape = (1, 16, 16, 24)
    rng = np.random.default_rng(53)
    net = U.UNet(shape, seed=4)
    net.set_params(_net_params(net.u, 8))
    d, h, w = 13, 11, 20
    dose, rho, _ = _net_inputs(rng, (d, h, w))
    td, tr = torch.from_numpy(dose).cuda(), torch.from_numpy(rho).cuda()
    out_r = torch.zeros((d, h, w), dtype=torch.float32, device="cuda")
    net.forward_region(td, tr, out_r)
    pd_ = torch.zeros(shape, dtype=torch.float32, device="cuda")
    pr = torch.zeros_like(pd_)
    pd_[0, :d, :h, :w] = td
    pr[0, :d, :h, :w] = tr
    out_f = torch.zeros_like(pd_)
    net.forward(pd_, pr, out_f)
    torch.cuda.synchronize()
    assert torch.equal(out_r, out_f[0, :d, :h, :w])
    with pytest.raises(ValueError):
        net.forward_region(torch.zeros((17, 4, 4), device="cuda"), torch.zeros((17, 4, 4), device="cuda"),
                           torch.zeros((17, 4, 4), device="cuda"))
    net.close()


def test_grad_norm_and_scaled_adam():
    """The device gradient norm equals the norm of the gradient read back,
    and two Adam steps on scaled gradients (the clipping factor) match the
    oracle's two steps on the same gradients and factors."""
    import torch
    _say("case: gradient norm and scaled adam")
    U = _unet()
    shape = (1, 8, 8, 16)
    rng = np.random.default_rng(37)
    net = U.UNet(shape, seed=5)
    p0 = _net_params(net.u, 6)
    net.set_params(p0)
    dose, rho, target = _net_inputs(rng, shape)
    td, tr, tt = (torch.from_numpy(a).cuda() for a in (dose, rho, target))
    orc = D.UNetOracle(p0.astype(np.float64))
    m1 = m2 = None
    lr = 1e-3
    for step, scale in ((1, 0.25), (2, 1.0)):
        net.backward(td, tr, tt)
        g = net.grads().astype(np.float64)
        norm = net.grad_norm()
        assert abs(norm - np.linalg.norm(g)) <= 1e-6 * np.linalg.norm(g)
        net.adam_step(lr, grad_scale=scale)
        if m1 is None:
            m1, m2 = np.zeros_like(g), np.zeros_like(g)
        m1, m2 = orc.adam_step(g, m1, m2, step, lr, grad_scale=scale)
    torch.cuda.synchronize()
    p2 = net.params().astype(np.float64)
    # the second step's gradients come from the GPU's own (FP32) first-step
    # parameters, which the oracle shares through g: compare the update
    dev = np.abs(p2 - orc.params)
    assert np.all(dev <= 1e-5 * lr + 2.0 ** -22 * np.abs(orc.params)), float(dev.max())
    net.close()


def test_training_reduces_loss():
    import torch
    _say("case: training loop")
    U = _unet()
    shape = (1, 16, 16, 16)
    rng = np.random.default_rng(41)
    net = U.UNet(shape, seed=7)
    dose, rho, _ = _net_inputs(rng, shape)
    # a target the network can represent: 1.1 dose + 0.05 max(dose) density
    target = (1.1 * dose + 0.05 * dose.max() * rho).astype(np.float32)
    td, tr, tt = (torch.from_numpy(a).cuda() for a in (dose, rho, target))
    first = net.backward(td, tr, tt)
    net.adam_step(1e-3)
    for _ in range(40):
        last = net.backward(td, tr, tt)
        net.adam_step(1e-3)
    _say("loss %.4e -> %.4e" % (first, last))
    assert np.isfinite(last) and last < 0.5 * first
    net.close()


def test_unet_max_size_runs():
    """The full 160x128x128 single-volume network: forward and backward run,
    the output is finite and the loss matches the oracle's on the same
    parameters within the network tolerance."""
    import torch
    _say("case: full-size network")
    U = _unet()
    shape = (1, 160, 128, 128)
    rng = np.random.default_rng(51)
    net = U.UNet(shape, seed=8)
    dose, rho, target = _net_inputs(rng, shape)
    td, tr, tt = (torch.from_numpy(a).cuda() for a in (dose, rho, target))
    out = torch.zeros_like(td)
    net.forward(td, tr, out)
    loss = net.backward(td, tr, tt)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    p = net.params().astype(np.float64)
    loss_o = D.UNetOracle(p).loss(dose.astype(np.float64), rho, target)
    _say("full-size loss gpu %.6e oracle %.6e" % (loss, loss_o))
    assert abs(loss - loss_o) <= 2.0 ** -5 * loss_o
    net.close()


# ------------------------------------------------------------ gamma

def _gamma_pair(rng, shape, noise=0.02):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ref = np.exp(-((x - nx / 2) ** 2 + (y - ny / 2) ** 2) / (2 * (0.2 * nx) ** 2)) * (1 + 0.03 * z)
    ref = ref * (z < 0.8 * nz)
    ev = np.roll(ref, 1, axis=0) * (1 + noise * rng.normal(size=shape))
    return ref, np.maximum(ev, 0.0)


@pytest.mark.parametrize("params", [
    dict(dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1, search_cm=0.4, step_cm=0.1),
    dict(dose_frac=0.03, dta_cm=0.3, cutoff_frac=0.0, search_cm=0.6, step_cm=0.05),
])
def test_gamma_matches_oracle(params):
    import torch
    _say("case: gamma %s" % params)
    U = _unet()
    rng = np.random.default_rng(61)
    shape = (30, 18, 22) if params["step_cm"] >= 0.1 else (14, 10, 12)
    ref, ev = _gamma_pair(rng, shape)
    vox = (0.2, 0.25, 0.2)
    g_o, rate_o, n_o = D.gamma_index(ref, ev, vox, **params)
    gam = torch.zeros(shape, dtype=torch.float32, device="cuda")
    rate, n = U.pmc_gamma_index(torch.from_numpy(ref).cuda(), torch.from_numpy(ev).cuda(), vox,
                                gamma=gam, **params)
    g = gam.cpu().numpy().astype(np.float64)
    assert n == n_o
    below = g_o < 0
    assert np.all(g[below] == -1.0)
    assert np.all(np.abs(g[~below] - g_o[~below]) <= 1e-5 * np.maximum(1.0, g_o[~below]))
    clear = (~below) & (np.abs(g_o - 1.0) > 1e-4)
    assert np.array_equal(g[clear] <= 1.0, g_o[clear] <= 1.0)
    amb = int(((~below) & ~clear).sum())
    assert abs(rate - rate_o) <= amb / max(n_o, 1) + 1e-12
    _say("gamma pass gpu %.4f oracle %.4f (n %d)" % (rate, rate_o, n))


def test_gamma_full_size_sampled():
    """128x128x160 at the default criteria (2 %, 2 mm, 10 % cutoff, 6 mm
    search, 0.5 mm step): 400 sampled voxels against the oracle."""
    import torch
    _say("case: gamma full size")
    U = _unet()
    rng = np.random.default_rng(62)
    shape = (160, 128, 128)
    ref, ev = _gamma_pair(rng, shape)
    gam = torch.zeros(shape, dtype=torch.float32, device="cuda")
    rate, n = U.pmc_gamma_index(torch.from_numpy(ref).cuda(), torch.from_numpy(ev).cuda(),
                                (0.2, 0.2, 0.2), gamma=gam)
    g = gam.cpu().numpy()
    pts = np.stack([rng.integers(0, s, 400) for s in shape], axis=1)
    g_o, _, _ = D.gamma_index(ref, ev, (0.2, 0.2, 0.2), points=pts)
    for z, y, x in pts:
        o = g_o[z, y, x]
        if o < 0:
            assert g[z, y, x] == -1.0
        else:
            assert abs(g[z, y, x] - o) <= 1e-5 * max(1.0, o), (z, y, x, g[z, y, x], o)
    assert n == int((ref >= 0.1 * ref.max()).sum())
    _say("full-size gamma pass rate %.4f over %d voxels" % (rate, n))


@pytest.mark.parametrize("shape,k", [((160, 128, 128), 4.0), ((7, 9, 11), 2.5), ((1, 1, 1), 4.0)])
def test_disagreement_rule_matches_oracle(shape, k):
    """The fallback rule's fraction and count equal the oracle's exactly
    (both sides take every decision in FP64 on the same float32 inputs):
    a dose with a spread of values, a noisy denoised copy with a seeded set
    of larger departures, per-voxel variances including zeros and negative
    estimates; a full-size grid, a ragged small one, a single voxel."""
    import torch
    _say("case: disagreement %s k=%g" % (shape, k))
    U = _unet()
    rng = np.random.default_rng(71)
    mc = rng.gamma(2.0, 1.0, size=shape) * (rng.random(shape) < 0.7)
    var = (0.05 * mc) ** 2 * rng.uniform(0.5, 1.5, size=shape)
    var[rng.random(shape) < 0.01] = 0.0
    var[rng.random(shape) < 0.005] = -1e-6
    den = (mc + rng.normal(0.0, 1.0, size=shape) * np.sqrt(np.maximum(var, 0.0))).astype(np.float32)
    big = rng.random(shape) < 0.03
    den[big] += (8.0 * np.sqrt(np.maximum(var[big], 1e-12))).astype(np.float32)
    frac, n = U.pmc_denoise_disagreement(torch.from_numpy(den).cuda(), torch.from_numpy(mc).cuda(),
                                         torch.from_numpy(var).cuda(), 0.1, k)
    frac_o, n_o = D.disagreement(den, mc, var, 0.1, k)
    _say("fraction %.6f of %d (oracle %.6f of %d)" % (frac, n, frac_o, n_o))
    assert n == n_o and frac == frac_o


def test_mfma_probe_rate_is_plausible():
    """The matrix-core probe: a register-only BF16 MFMA stream over the whole
    device reaches a substantial part of the 2.5 PFLOP/s dense peak and never
    exceeds it."""
    U = _unet()
    ms, flop = U.pmc_nn_mfma_probe(4000)
    tflops = flop / (ms * 1e-3) / 1e12
    _say("MFMA probe: %.1f TFLOP/s (%.3f ms for %.3g FLOP)" % (tflops, ms, flop))
    assert 500.0 < tflops < 2600.0, tflops
