"""FP64 CPU oracle of the dose denoiser and of the 3-D gamma index.

Test infrastructure only: the test-suite, the smoke check and the
benchmark's CPU-baseline leg may use this module; the library never does.
It shares no code with the HIP path.

What it computes (the denoiser has no counterpart in the paper; the gamma
index is the evaluation tool the paper uses for its dose comparisons,
Sec. II.D, defined by Low et al.):

* ``conv3d`` / ``conv3d_backward_data`` / ``conv3d_backward_weight``: the
  3x3x3, stride-1, zero-padded cross-correlation and its two adjoints, as
  plain sums over the 27 taps (channels-last arrays, the weight matrix in the
  library's [cout][tap*cin + ci] order, tap = (kz*3 + ky)*3 + kx).
* ``UNetOracle``: the 4-level network (16/32/64/128 channels, one conv +
  leaky ReLU (slope 0.01) per level, 2x2x2 average pooling, nearest upsampling and concatenation
  [coarse, skip], 1x1x1 residual head scaled by max(dose)), its loss (the
  squared error in units of max(dose) summed over all voxels, divided by the
  number of voxels with dose >= 1% of max(dose)), the gradient by
  reverse-mode differentiation in FP64
  (PyTorch CPU autograd used as the differentiation primitive), and one Adam
  step (Kingma and Ba, beta1 0.9, beta2 0.999, eps 1e-8).
* ``gamma_index``: for each reference voxel at or above cutoff * max(ref),
  the minimum over the points of a cubic search grid inside a sphere of the
  combined distance / dose-difference metric, the evaluated dose taken by
  trilinear interpolation; points outside the grid are skipped.

Pins (tests/test_denoiser_oracle_pins.py): conv against an impulse response
and against torch.nn.functional.conv3d; both adjoints against the inner
product identity; the network gradient against central finite differences;
the residual head and the pooling pair against their closed forms; gamma
against identical and uniformly scaled distributions, against the closed
minimum for a shifted linear ramp, and against a pure-Python brute force.
"""
from __future__ import annotations

import numpy as np

# ------------------------------------------------------------ convolution


def _taps():
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                yield (kz * 3 + ky) * 3 + kx, (kz - 1, ky - 1, kx - 1)


def _shifted(x, off):
    """s[v] = x[v + off] with zeros outside (x: [n, d, h, w, c])."""
    n, d, h, w, c = x.shape
    s = np.zeros_like(x)
    oz, oy, ox = off
    zs, ys, xs = [slice(max(0, -o), min(L, L - o)) for o, L in zip(off, (d, h, w))]
    zt, yt, xt = [slice(max(0, o), min(L, L + o)) for o, L in zip(off, (d, h, w))]
    s[:, zs, ys, xs, :] = x[:, zt, yt, xt, :]
    return s


LEAK = 0.01   # negative slope of the activation after every convolution


def leaky_relu(y):
    """y if y > 0 else LEAK * y."""
    return np.where(y > 0.0, y, LEAK * y)


def conv3d(x, wmat, bias=None, relu=False):
    """y[v][co] = bias[co] + sum_{tap, ci} x[v + off(tap)][ci] * W[co][tap*cin + ci]."""
    x = np.asarray(x, np.float64)
    cin = x.shape[-1]
    wmat = np.asarray(wmat, np.float64)
    cout = wmat.shape[0]
    y = np.zeros(x.shape[:-1] + (cout,))
    for tap, off in _taps():
        wt = wmat[:, tap * cin:(tap + 1) * cin]          # [cout, cin]
        y += _shifted(x, off) @ wt.T
    if bias is not None:
        y += np.asarray(bias, np.float64)
    if relu:
        y = leaky_relu(y)
    return y


def conv3d_at(x, wmat, bias, points, relu=False):
    """The same convolution evaluated one output voxel at a time at
    ``points`` (list of (n, z, y, x)), for sampled checks on large grids."""
    x = np.asarray(x)
    n_, d, h, w, cin = x.shape
    wmat = np.asarray(wmat, np.float64)
    out = []
    for (n, z, yy, xx) in points:
        acc = np.zeros(wmat.shape[0]) if bias is None else np.asarray(bias, np.float64).copy()
        for tap, (oz, oy, ox) in _taps():
            zz, y2, x2 = z + oz, yy + oy, xx + ox
            if 0 <= zz < d and 0 <= y2 < h and 0 <= x2 < w:
                acc += wmat[:, tap * cin:(tap + 1) * cin] @ x[n, zz, y2, x2].astype(np.float64)
        out.append(leaky_relu(acc) if relu else acc)
    return np.array(out)


def conv3d_backward_data(dy, wmat, cin):
    """dx[v][ci] = sum_{tap, co} dy[v - off(tap)][co] * W[co][tap*cin + ci]
    (the adjoint of conv3d in its input)."""
    dy = np.asarray(dy, np.float64)
    wmat = np.asarray(wmat, np.float64)
    dx = np.zeros(dy.shape[:-1] + (cin,))
    for tap, off in _taps():
        wt = wmat[:, tap * cin:(tap + 1) * cin]          # [cout, cin]
        dx += _shifted(dy, tuple(-o for o in off)) @ wt
    return dx


def conv3d_backward_weight(x, dy, kp):
    """dW[co][tap*cin + ci] = sum_v dy[v][co] * x[v + off(tap)][ci]
    (the adjoint of conv3d in its weights); columns beyond 27*cin are 0."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    cin, cout = x.shape[-1], dy.shape[-1]
    dw = np.zeros((cout, kp))
    dyf = dy.reshape(-1, cout)
    for tap, off in _taps():
        dw[:, tap * cin:(tap + 1) * cin] = dyf.T @ _shifted(x, off).reshape(-1, cin)
    return dw


def pool_avg(x):
    """2x2x2 average pooling, channels-last."""
    n, d, h, w, c = x.shape
    return np.asarray(x, np.float64).reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def upsample_nearest(x):
    """Nearest-neighbour 2x upsampling, channels-last."""
    x = np.asarray(x, np.float64)
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


# ------------------------------------------------------------ network

CONVS = ((8, 16), (16, 32), (32, 64), (64, 128), (192, 64), (96, 32), (48, 16))
NAMES = ("enc1", "enc2", "enc3", "enc4", "dec3", "dec2", "dec1")


def kp(cin):
    return (27 * cin + 31) // 32 * 32


def param_layout():
    """[(name, offset of W, offset of b, cin, cout, Kp)], head w offset,
    head b offset, total length: the library's flat parameter order."""
    out, off = [], 0
    for name, (cin, cout) in zip(NAMES, CONVS):
        k = kp(cin)
        out.append((name, off, off + cout * k, cin, cout, k))
        off += cout * k + cout
    return out, off, off + 16, off + 17


def _torch_weight(torch, wmat, cin, cout):
    # [cout][tap*cin + ci] -> [cout][ci][kz][ky][kx]
    w = wmat[:, :27 * cin].reshape(cout, 3, 3, 3, cin)
    return w.permute(0, 4, 1, 2, 3)


class UNetOracle:
    """FP64 forward, loss and gradient of the denoiser for one parameter
    vector (the library's flat layout)."""

    def __init__(self, params):
        self.params = np.asarray(params, np.float64).copy()
        self.layout, self.off_hw, self.off_hb, self.n = param_layout()
        assert self.params.size == self.n

    def _graph(self, dose, rho, target=None, need_grad=False):
        import torch
        F = torch.nn.functional
        p = torch.tensor(self.params, dtype=torch.float64, requires_grad=need_grad)
        dose_t = torch.tensor(np.asarray(dose, np.float64))        # [n, d, h, w]
        rho_t = torch.tensor(np.asarray(rho, np.float64))
        scale = dose_t.max()
        n, d, h, w = dose_t.shape
        x = torch.zeros((n, 8, d, h, w), dtype=torch.float64)
        x = torch.cat([(dose_t / scale)[:, None], (rho_t * 0.5)[:, None], x[:, 2:]], dim=1)

        def conv(name, inp):
            _, ow, ob, cin, cout, k = next(l for l in self.layout if l[0] == name)
            wmat = p[ow:ow + cout * k].reshape(cout, k)
            wt = _torch_weight(torch, wmat, cin, cout)
            return F.leaky_relu(F.conv3d(inp, wt, p[ob:ob + cout], padding=1), LEAK)

        def up_cat(coarse, skip):
            return torch.cat([coarse.repeat_interleave(2, 2).repeat_interleave(2, 3)
                              .repeat_interleave(2, 4), skip], dim=1)

        e1 = conv("enc1", x)
        e2 = conv("enc2", F.avg_pool3d(e1, 2))
        e3 = conv("enc3", F.avg_pool3d(e2, 2))
        e4 = conv("enc4", F.avg_pool3d(e3, 2))
        d3 = conv("dec3", up_cat(e4, e3))
        d2 = conv("dec2", up_cat(d3, e2))
        d1 = conv("dec1", up_cat(d2, e1))
        head = torch.einsum("ncdhw,c->ndhw", d1, p[self.off_hw:self.off_hw + 16]) + p[self.off_hb]
        out = dose_t + scale * head
        loss = None
        if target is not None:
            t = torch.tensor(np.asarray(target, np.float64))
            n_region = max(1, int((dose_t >= 0.01 * scale).sum()))
            loss = (((out - t) / scale) ** 2).sum() / n_region
        return p, out, loss

    def forward(self, dose, rho):
        _, out, _ = self._graph(dose, rho)
        return out.detach().numpy()

    def loss(self, dose, rho, target):
        _, _, l = self._graph(dose, rho, target)
        return float(l)

    def loss_and_grad(self, dose, rho, target):
        p, out, l = self._graph(dose, rho, target, need_grad=True)
        l.backward()
        return float(l.detach()), p.grad.numpy().copy(), out.detach().numpy()

    def adam_step(self, grad, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8, grad_scale=1.0):
        """One Adam step on grad_scale * grad (the caller's clipping factor)
        for the held parameters; returns the new moments."""
        grad = grad_scale * grad
        m1 = b1 * m1 + (1 - b1) * grad
        m2 = b2 * m2 + (1 - b2) * grad * grad
        mh = m1 / (1 - b1 ** step)
        vh = m2 / (1 - b2 ** step)
        self.params = self.params - lr * mh / (np.sqrt(vh) + eps)
        return m1, m2


# ------------------------------------------------------------ gamma index


def _trilinear(ev, pz, py, px):
    nz, ny, nx = ev.shape
    z0 = np.minimum(np.floor(pz).astype(np.int64), nz - 1)
    y0 = np.minimum(np.floor(py).astype(np.int64), ny - 1)
    x0 = np.minimum(np.floor(px).astype(np.int64), nx - 1)
    z1, y1, x1 = np.minimum(z0 + 1, nz - 1), np.minimum(y0 + 1, ny - 1), np.minimum(x0 + 1, nx - 1)
    tz, ty, tx = pz - z0, py - y0, px - x0
    val = 0.0
    for zc, wz in ((z0, 1 - tz), (z1, tz)):
        for yc, wy in ((y0, 1 - ty), (y1, ty)):
            for xc, wx in ((x0, 1 - tx), (x1, tx)):
                val = val + ev[zc, yc, xc] * wz * wy * wx
    return val


def search_offsets(search_cm, step_cm):
    """Offsets (cm) of the cubic search grid that lie inside the sphere."""
    m = int(np.floor(search_cm / step_cm + 1e-4))
    out = []
    for k in range(-m, m + 1):
        for j in range(-m, m + 1):
            for i in range(-m, m + 1):
                o = np.array([k, j, i], np.float64) * step_cm
                if (o * o).sum() <= search_cm * search_cm * (1 + 1e-6):
                    out.append(o)
    return out


def gamma_index(ref, ev, voxel_cm, dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1, search_cm=0.6,
                step_cm=0.05, points=None):
    """Gamma of ``ev`` against ``ref`` ([nz, ny, nx]); voxel_cm = (dx, dy, dz).
    Returns (gamma array with -1 below the cutoff, pass rate, count).  With
    ``points`` (an [m, 3] array of (z, y, x)) only those voxels are evaluated
    (the others read -1)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    nz, ny, nx = ref.shape
    dx, dy, dz = voxel_cm
    dmax = ref.max()
    crit = dose_frac * dmax
    mask = ref >= cutoff_frac * dmax
    if points is not None:
        sel = np.zeros_like(mask)
        pts = np.asarray(points)
        sel[pts[:, 0], pts[:, 1], pts[:, 2]] = True
        mask &= sel
    zz, yy, xx = np.nonzero(mask)
    r = ref[mask]
    best = np.full(r.shape, np.inf)
    for oz, oy, ox in search_offsets(search_cm, step_cm):
        pz, py, px = zz + oz / dz, yy + oy / dy, xx + ox / dx
        inside = (pz >= 0) & (py >= 0) & (px >= 0) & (pz <= nz - 1) & (py <= ny - 1) & (px <= nx - 1)
        val = _trilinear(ev, np.clip(pz, 0, nz - 1), np.clip(py, 0, ny - 1), np.clip(px, 0, nx - 1))
        g2 = (oz * oz + oy * oy + ox * ox) / dta_cm ** 2 + ((val - r) / crit) ** 2
        best = np.where(inside, np.minimum(best, g2), best)
    g = np.full(ref.shape, -1.0)
    g[mask] = np.sqrt(best)
    n = int(mask.sum())
    rate = float((g[mask] <= 1.0).mean()) if n else 1.0
    return g, rate, n


def disagreement(den, mc, var, cutoff_frac=0.1, k_sigma=4.0):
    """The denoiser's fallback rule written out: among the voxels with
    mc >= cutoff_frac * max(mc) and mc > 0, the fraction where
    |den - mc| > k_sigma * sqrt(max(var, 0)), i.e. where the denoised dose
    departs from the Monte Carlo dose it was computed from by more than
    k_sigma of that dose's own standard error (the 10-group estimate of
    Eq. 5).  cutoff_frac and k_sigma are taken at float32 precision (as the
    library receives them), den as float32 values.  Returns (fraction,
    number of voxels above the cutoff)."""
    c = float(np.float32(cutoff_frac))
    k = float(np.float32(k_sigma))
    den = np.asarray(den, np.float32).astype(np.float64).ravel()
    mc = np.asarray(mc, np.float64).ravel()
    var = np.asarray(var, np.float64).ravel()
    thr = c * mc.max() if mc.size else 0.0
    sel = (mc >= thr) & (mc > 0.0)
    n = int(sel.sum())
    if n == 0:
        return 0.0, 0
    off = np.abs(den[sel] - mc[sel]) > k * np.sqrt(np.maximum(var[sel], 0.0))
    return float(off.sum()) / n, n
