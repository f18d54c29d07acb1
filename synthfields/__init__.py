"""Seeded synthetic 2D time-varying vector fields.

These stand in for the paper's simulation datasets (cylinder flows, a fluid
ensemble, decaying turbulence), which are not available here.  The module
holds no compressor arithmetic: it only makes input data, shared by the
oracle tests, the GPU tests and the benchmark.

Every generator returns ``(field, meta)``: ``field`` is a float32 tensor of
shape (2, T, H, W) (u plane then v plane, x fastest) and ``meta`` a dict with
at least ``dt_dx`` (time step over grid spacing, i.e. cells per step per unit
velocity), ``eb`` and the recipe parameters.

Recipes
-------
workload 0  64x64x8, four Lamb-Oseen vortices (core radius U(3,6) cells,
            circulation +-U(0.5,2)) translating at <= 0.5 cell/step, plus
            N(0,1e-3) noise; dt_dx = 1.
workload 1  720x1440x64 lat-lon-like wind: divergence-free random field from a
            streamfunction with |psi_hat| ~ k^-3 (rms 10), plus a zonal jet
            20 exp(-(y-360)^2 / (2 60^2)); each step the random part is
            advected semi-Lagrangianly by the total wind (CFL 0.5, periodic x)
            and refreshed with 1 % new spectral forcing.
workload 2  2048x2048x32 turbulence-like: streamfunction with E(k) ~ k^-5/3
            for 4 <= |k| <= 512 (rms 1), self-advected at CFL 0.5 and
            re-projected divergence-free each step, plus 64 translating
            Lamb-Oseen vortices with circulation scaled by the rms.
workload 3  256 fields: side round(exp U(ln 64, ln 1024)), T uniform in 8..64,
            4..32 vortices as workload 0.
workload 4  1024x1024x128 as workload 2 with another seed.
workload 5  1024x1024x64 as workload 2 (another seed, 16 vortices) with the
            time step raised to CFL 6: the fastest point moves 6 cells per
            step, so backtraces of 1, 2 and 4 cells per step differ.
"""
import math

import numpy as np
import torch


def _lamb_oseen_add(u, v, X, Y, cx, cy, gamma, rc):
    """Add one Lamb-Oseen swirl centred at (cx, cy): v_theta(r) =
    gamma / (2 pi r) (1 - exp(-r^2/rc^2)); no translation velocity is added,
    so an isolated vortex's critical point is its centre."""
    dx = X - cx
    dy = Y - cy
    r2 = dx * dx + dy * dy
    s = r2 / (rc * rc)
    # (1 - exp(-s)) / r^2, with the limit 1/rc^2 at the centre
    g = torch.where(s > 1e-12, -torch.expm1(-s) / torch.clamp(r2, min=1e-300),
                    torch.full_like(r2, 1.0 / (rc * rc)))
    g = g * (gamma / (2.0 * math.pi))
    u -= dy * g
    v += dx * g


def vortex_params(n, H, W, rng, margin=8.0, rc=(3.0, 6.0), gamma=(0.5, 2.0), speed=0.5):
    """Centres, velocities (cells/step), circulations and core radii."""
    mx = min(margin, (W - 1) / 4.0)
    my = min(margin, (H - 1) / 4.0)
    c0 = np.stack([rng.uniform(mx, W - 1 - mx, n), rng.uniform(my, H - 1 - my, n)], 1)
    ang = rng.uniform(0.0, 2.0 * math.pi, n)
    sp = rng.uniform(0.0, speed, n)
    vel = np.stack([sp * np.cos(ang), sp * np.sin(ang)], 1)
    gam = rng.uniform(gamma[0], gamma[1], n) * rng.choice([-1.0, 1.0], n)
    r = rng.uniform(rc[0], rc[1], n)
    return c0, vel, gam, r


def vortex_field(H, W, T, n_vortices, seed, noise=1e-3, device="cpu", params=None,
                 gamma_scale=1.0, dtype=torch.float64):
    """Sum of translating Lamb-Oseen vortices plus Gaussian noise."""
    rng = np.random.default_rng(seed)
    if params is None:
        params = vortex_params(n_vortices, H, W, rng)
    c0, vel, gam, rc = params
    ys = torch.arange(H, dtype=dtype, device=device).view(H, 1)
    xs = torch.arange(W, dtype=dtype, device=device).view(1, W)
    X = xs.expand(H, W)
    Y = ys.expand(H, W)
    out = torch.empty((2, T, H, W), dtype=torch.float32, device=device)
    for t in range(T):
        u = torch.zeros((H, W), dtype=dtype, device=device)
        v = torch.zeros((H, W), dtype=dtype, device=device)
        for i in range(len(gam)):
            cx = c0[i, 0] + vel[i, 0] * t
            cy = c0[i, 1] + vel[i, 1] * t
            _lamb_oseen_add(u, v, X, Y, float(cx), float(cy), float(gam[i]) * gamma_scale, float(rc[i]))
        out[0, t] = u.to(torch.float32)
        out[1, t] = v.to(torch.float32)
    if noise > 0:
        g = torch.Generator().manual_seed(int(seed) + 7919)
        nz = torch.randn((2, T, H, W), generator=g, dtype=torch.float32) * noise
        out += nz.to(device)
    meta = dict(dt_dx=1.0, c0=c0, vel=vel, gamma=gam, rc=rc, seed=seed)
    return out, meta


def _spectral_psi(H, W, slope, kmin, kmax, gen, device):
    """Random streamfunction with |psi_hat(k)| = k^slope on kmin <= |k| <= kmax."""
    ky = torch.fft.fftfreq(H, d=1.0 / H).view(H, 1)
    kx = torch.fft.rfftfreq(W, d=1.0 / W).view(1, W // 2 + 1)
    k = torch.sqrt(kx * kx + ky * ky)
    amp = torch.where((k >= kmin) & (k <= kmax), torch.clamp(k, min=1e-9) ** slope,
                      torch.zeros_like(k))
    ph = torch.rand((H, W // 2 + 1), generator=gen, dtype=torch.float64) * (2 * math.pi)
    spec = (amp * torch.exp(1j * ph)).to(torch.complex128)
    return spec.to(device)


def _velocity_from_psi_hat(ph, H, W):
    ky = torch.fft.fftfreq(H, d=1.0 / H).view(H, 1).to(ph.device) * (2 * math.pi / H)
    kx = torch.fft.rfftfreq(W, d=1.0 / W).view(1, -1).to(ph.device) * (2 * math.pi / W)
    u = torch.fft.irfft2(-1j * ky * ph, s=(H, W))
    v = torch.fft.irfft2(1j * kx * ph, s=(H, W))
    return u, v


def _project(u, v):
    """Remove the divergent part of (u, v) with an FFT projection."""
    H, W = u.shape
    ky = torch.fft.fftfreq(H, d=1.0 / H).view(H, 1).to(u.device) * (2 * math.pi / H)
    kx = torch.fft.rfftfreq(W, d=1.0 / W).view(1, -1).to(u.device) * (2 * math.pi / W)
    U = torch.fft.rfft2(u)
    V = torch.fft.rfft2(v)
    k2 = kx * kx + ky * ky
    k2[0, 0] = 1.0
    dv = (kx * U + ky * V) / k2
    U = U - kx * dv
    V = V - ky * dv
    return torch.fft.irfft2(U, s=(H, W)), torch.fft.irfft2(V, s=(H, W))


def _bilinear(f, px, py, periodic_x):
    H, W = f.shape
    if periodic_x:
        px = torch.remainder(px, W)
    else:
        px = px.clamp(0, W - 1)
    py = py.clamp(0, H - 1)
    x0 = torch.floor(px)
    y0 = torch.floor(py)
    fx = px - x0
    fy = py - y0
    x0 = x0.long()
    y0 = y0.long()
    if periodic_x:
        x0 = x0 % W
        x1 = (x0 + 1) % W
    else:
        x1 = torch.clamp(x0 + 1, max=W - 1)
    y1 = torch.clamp(y0 + 1, max=H - 1)
    a = f[y0, x0]
    b = f[y0, x1]
    c = f[y1, x0]
    d = f[y1, x1]
    return a * (1 - fx) * (1 - fy) + b * fx * (1 - fy) + c * (1 - fx) * fy + d * fx * fy


def _advect(u, v, au, av, dt, periodic_x):
    """Semi-Lagrangian advection of (u, v) by the wind (au, av) over dt."""
    H, W = u.shape
    ys = torch.arange(H, dtype=u.dtype, device=u.device).view(H, 1).expand(H, W)
    xs = torch.arange(W, dtype=u.dtype, device=u.device).view(1, W).expand(H, W)
    px = xs - dt * au
    py = ys - dt * av
    return _bilinear(u, px, py, periodic_x), _bilinear(v, px, py, periodic_x)


def _rms(u, v):
    return float(torch.sqrt(torch.mean(u * u + v * v) / 2))


def wind_field(H=720, W=1440, T=64, seed=1000, device="cpu", dtype=torch.float64):
    """Workload 1 recipe (lat-lon-like wind)."""
    gen = torch.Generator().manual_seed(seed)
    ph = _spectral_psi(H, W, -3.0, 1.0, max(H, W), gen, device)
    ru, rv = _velocity_from_psi_hat(ph, H, W)
    s = 10.0 / max(_rms(ru, rv), 1e-30)
    ru, rv = ru * s, rv * s
    y = torch.arange(H, dtype=dtype, device=device).view(H, 1)
    y0 = H / 2.0
    jet = (20.0 * torch.exp(-((y - y0) ** 2) / (2 * 60.0 ** 2))).expand(H, W)
    umax = float(torch.max(torch.abs(ru + jet)).item())
    vmax = float(torch.max(torch.abs(rv)).item())
    dt = 0.5 / max(umax, vmax, 1e-30)
    out = torch.empty((2, T, H, W), dtype=torch.float32, device=device)
    for t in range(T):
        out[0, t] = (ru + jet).to(torch.float32)
        out[1, t] = rv.to(torch.float32)
        if t + 1 < T:
            au, av = ru + jet, rv
            nu, nv = _advect(ru, rv, au, av, dt, periodic_x=True)
            fu, fv = _velocity_from_psi_hat(_spectral_psi(H, W, -3.0, 1.0, max(H, W), gen, device), H, W)
            fs = 10.0 / max(_rms(fu, fv), 1e-30)
            ru = math.sqrt(0.99) * nu + math.sqrt(0.01) * fu * fs
            rv = math.sqrt(0.99) * nv + math.sqrt(0.01) * fv * fs
    return out, dict(dt_dx=dt, seed=seed)


def turbulence_field(H=2048, W=2048, T=32, seed=2000, n_vortices=64, device="cpu",
                     dtype=torch.float64, cfl=0.5):
    """Workload 2/4/5 recipe (self-advected k^-5/3 turbulence plus vortices);
    the time step moves the fastest point cfl cells per step."""
    gen = torch.Generator().manual_seed(seed)
    kmax = min(512.0, min(H, W) / 2.0)
    ph = _spectral_psi(H, W, -7.0 / 3.0, 4.0, kmax, gen, device)
    u, v = _velocity_from_psi_hat(ph, H, W)
    s = 1.0 / max(_rms(u, v), 1e-30)
    u, v = u * s, v * s
    rng = np.random.default_rng(seed)
    vp = vortex_params(n_vortices, H, W, rng, margin=16.0)
    vort, _ = vortex_field(H, W, T, n_vortices, seed, noise=0.0, device=device, params=vp,
                           gamma_scale=1.0, dtype=dtype)
    umax = float(torch.max(torch.abs(u)).item()) + 1e-30
    vmax = float(torch.max(torch.abs(v)).item()) + 1e-30
    dt = cfl / max(umax, vmax)
    out = torch.empty((2, T, H, W), dtype=torch.float32, device=device)
    for t in range(T):
        out[0, t] = u.to(torch.float32) + vort[0, t]
        out[1, t] = v.to(torch.float32) + vort[1, t]
        if t + 1 < T:
            u, v = _advect(u, v, u, v, dt, periodic_x=True)
            u, v = _project(u, v)
    return out, dict(dt_dx=dt, seed=seed, cfl=cfl)


WORKLOADS = {
    0: dict(shape=(64, 64, 8), eb=1e-2, predictor=2, mode_bt=1),
    1: dict(shape=(720, 1440, 64), eb=1e-3, predictor=2, mode_bt=1),
    2: dict(shape=(2048, 2048, 32), eb=1e-3, predictor=2, mode_bt=1),
    4: dict(shape=(1024, 1024, 128), eb=1e-3, predictor=3, mode_bt=4),
    5: dict(shape=(1024, 1024, 64), eb=1e-3, predictor=3, mode_bt=4),
}


def workload(cfg, index=0, device="cpu", shape=None):
    """Field of workload ``cfg`` (seed 1000*cfg + index), optionally at another
    (H, W, T) shape with the same recipe (used for crops of the big ones)."""
    seed = 1000 * cfg + index
    if cfg in (0, 3):
        H, W, T = shape or (64, 64, 8)
        rng = np.random.default_rng(seed)
        nv = 4 if cfg == 0 else int(rng.integers(4, 33))
        f, m = vortex_field(H, W, T, nv, seed, device=device)
    elif cfg == 1:
        H, W, T = shape or WORKLOADS[1]["shape"]
        f, m = wind_field(H, W, T, seed, device=device)
    elif cfg in (2, 4):
        H, W, T = shape or WORKLOADS[cfg]["shape"]
        nv = 64 if min(H, W) >= 256 else 8
        f, m = turbulence_field(H, W, T, seed, n_vortices=nv, device=device)
    elif cfg == 5:
        H, W, T = shape or WORKLOADS[cfg]["shape"]
        f, m = turbulence_field(H, W, T, seed, n_vortices=16, device=device, cfl=6.0)
    else:
        raise ValueError("unknown workload %r" % cfg)
    m = dict(m)
    if cfg in WORKLOADS:
        m.update(eb=WORKLOADS[cfg]["eb"], predictor=WORKLOADS[cfg]["predictor"],
                 mode_bt=WORKLOADS[cfg]["mode_bt"])
    else:
        m.update(eb=1e-2, predictor=2, mode_bt=1)
    return f, m


def spiked_field(H=96, W=128, T=8, frac=0.01, amp=0.1, seed=11):
    """A smooth (affine) field with a fraction `frac` of its components
    displaced by U(-amp, amp): residual codes concentrate on a few symbols
    with a long tail of rare ones, whose Huffman codewords exceed 12 bits."""
    rng = np.random.default_rng(seed)
    t, y, x = np.meshgrid(np.arange(T), np.arange(H), np.arange(W), indexing="ij")
    f = np.stack([0.5 + 0.001 * x + 0.002 * y + 0.003 * t, -0.3 + 0.002 * x - 0.001 * y + 0.001 * t])
    f = f.astype(np.float32)
    m = rng.random(f.shape) < frac
    f[m] += rng.uniform(-amp, amp, int(m.sum())).astype(np.float32)
    return torch.from_numpy(f), dict(dt_dx=1.0, seed=seed)


def batch_shapes(n=256, seed=3000):
    """(H, W, T) of the uneven batch: side log-uniform in [64, 1024], T in 8..64."""
    rng = np.random.default_rng(seed)
    sides = np.round(np.exp(rng.uniform(math.log(64), math.log(1024), n))).astype(int)
    ts = rng.integers(8, 65, n)
    return [(int(s), int(s), int(t)) for s, t in zip(sides, ts)]


def batch_field(i, shape, device="cpu"):
    """Field i of the uneven batch (vortex recipe, 4..32 vortices)."""
    H, W, T = shape
    seed = 3000 + i
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(4, 33))
    f, m = vortex_field(H, W, T, nv, seed, device=device)
    m.update(eb=1e-2, predictor=2, mode_bt=1)
    return f, m
