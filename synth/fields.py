"""Seeded synthetic stand-ins for the paper's SDRBench fields.

The paper evaluates on Hurricane, CESM-ATM, SCALE-LETKF and Miranda
(Sec. VI-A, Table III); none of them is available here, so every input is a
seeded random field with a comparable structure:

* ``sinusoid_1d``   -- 1-D sum of 8 sinusoids (periods 64..65536) plus noise.
* ``grf_3d``        -- 3-D Gaussian random field whose shell energy spectrum
                       falls as k^-5/3 (turbulence-like, like Miranda).
* ``climate_steps`` -- 2-D lat/lon climate-like steps (like CESM-ATM): smooth
                       latitude-dependent mean, k^-5/3 noise, AR(1) in time,
                       and a 2 % land mask of exact zeros (``climate_steps_device``:
                       the same recipe built on a GPU for the 100-step sweep).
* ``batch_specs`` / ``batch_field`` -- thousands of smooth-plus-noise fields of
                       log-uniform size and mixed dimensionality.

Everything is float32 on output; intermediate arithmetic is float64 (numpy) or
float32 complex FFTs (torch, for the large 3-D field on a device).
"""
import math

import numpy as np


def value_range(x) -> float:
    """max - min of a field in float64 (numpy array or torch tensor)."""
    if hasattr(x, "detach"):
        return float(x.max().double().item() - x.min().double().item())
    x = np.asarray(x)
    return float(np.float64(x.max()) - np.float64(x.min()))


def rel_eb(x, rel: float) -> float:
    """Absolute error bound equal to `rel` times the field's value range."""
    r = value_range(x)
    return rel * r if r > 0 else rel


def sinusoid_1d(n: int = 1 << 20, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5, size=8)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=8)
    periods = 64.0 * 1024.0 ** (np.arange(8) / 7.0)
    i = np.arange(n, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    for a, p, t in zip(amp, phase, periods):
        y += a * np.sin(2.0 * math.pi * i / t + p)
    y += rng.normal(0.0, 1e-3 * (y.max() - y.min()), size=n)
    return y.astype(np.float32)


def _radial_k(shape, real_last=True):
    """|k| in integer wavenumbers on an rfft grid (numpy)."""
    axes = []
    for d, m in enumerate(shape):
        if real_last and d == len(shape) - 1:
            axes.append(np.fft.rfftfreq(m) * m)
        else:
            axes.append(np.fft.fftfreq(m) * m)
    grids = np.meshgrid(*axes, indexing="ij", sparse=True)
    k2 = sum(g * g for g in grids)
    return np.sqrt(k2)


def grf_3d(n: int = 512, seed: int = 3, device=None):
    """n^3 Gaussian random field with E(k) ~ k^-5/3, unit std, float32.

    White noise is filtered by |k|^(-11/6) in Fourier space (the amplitude
    whose shell-integrated energy spectrum falls as k^-5/3); k = 0 is removed.
    With ``device`` (a torch device) the field is built there with torch and
    returned as a torch tensor; otherwise numpy is used.
    """
    if device is not None:
        import torch

        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        white = torch.randn((n, n, n), generator=gen, device=device, dtype=torch.float32)
        spec = torch.fft.rfftn(white)
        del white
        f = torch.fft.fftfreq(n, device=device) * n
        fr = torch.fft.rfftfreq(n, device=device) * n
        k2 = f.view(n, 1, 1) ** 2 + f.view(1, n, 1) ** 2 + fr.view(1, 1, -1) ** 2
        k2[0, 0, 0] = 1.0
        filt = k2.pow(-11.0 / 12.0)
        filt[0, 0, 0] = 0.0
        spec.mul_(filt)
        del k2, filt
        field = torch.fft.irfftn(spec, s=(n, n, n))
        del spec
        field = (field - field.mean()) / field.std()
        return field.to(torch.float32).contiguous()
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    spec = np.fft.rfftn(white)
    k = _radial_k((n, n, n))
    with np.errstate(divide="ignore"):
        filt = np.where(k > 0, k ** (-11.0 / 6.0), 0.0)
    field = np.fft.irfftn(spec * filt, s=(n, n, n), axes=(0, 1, 2))
    field = (field - field.mean()) / field.std()
    return field.astype(np.float32)


def _grf_2d(ny, nx, rng, amp_exponent):
    white = rng.standard_normal((ny, nx))
    k = _radial_k((ny, nx))
    with np.errstate(divide="ignore"):
        filt = np.where(k > 0, k ** amp_exponent, 0.0)
    f = np.fft.irfft2(np.fft.rfft2(white) * filt, s=(ny, nx))
    return (f - f.mean()) / f.std()


def climate_steps(nsteps: int = 100, ny: int = 1800, nx: int = 3600, seed: int = 5,
                  mask_seed: int = 6, rho: float = 0.95):
    """Yield `nsteps` float32 (ny, nx) climate-like steps, longitude fastest.

    step_t = 250 + 40 cos^2(lat) + 5 * noise_t, with noise_t an AR(1) sequence
    (coefficient `rho`) of 2-D fields whose energy spectrum falls as k^-5/3
    (amplitude |k|^-4/3); 2 % of the cells (a fixed smooth mask, the top 2 %
    of a |k|^-3 field) are exactly 0.0.
    """
    lat = np.linspace(-0.5 * math.pi, 0.5 * math.pi, ny)
    mu = (250.0 + 40.0 * np.cos(lat) ** 2)[:, None]
    mrng = np.random.default_rng(mask_seed)
    smooth = _grf_2d(ny, nx, mrng, -3.0)
    land = smooth >= np.quantile(smooth, 0.98)
    rng = np.random.default_rng(seed)
    noise = _grf_2d(ny, nx, rng, -4.0 / 3.0)
    scale = math.sqrt(1.0 - rho * rho)
    for t in range(nsteps):
        if t > 0:
            noise = rho * noise + scale * _grf_2d(ny, nx, rng, -4.0 / 3.0)
        step = mu + 5.0 * noise
        step[land] = 0.0
        yield step.astype(np.float32)


def _grf_2d_device(ny, nx, gen, amp_exponent, device):
    import torch

    white = torch.randn((ny, nx), generator=gen, device=device, dtype=torch.float64)
    fy = torch.fft.fftfreq(ny, device=device, dtype=torch.float64) * ny
    fx = torch.fft.rfftfreq(nx, device=device, dtype=torch.float64) * nx
    k2 = fy.view(ny, 1) ** 2 + fx.view(1, -1) ** 2
    k2[0, 0] = 1.0
    filt = k2.pow(0.5 * amp_exponent)
    filt[0, 0] = 0.0
    f = torch.fft.irfft2(torch.fft.rfft2(white) * filt, s=(ny, nx))
    return (f - f.mean()) / f.std()


def climate_steps_device(nsteps: int = 100, ny: int = 1800, nx: int = 3600, seed: int = 5,
                         mask_seed: int = 6, rho: float = 0.95, device=None):
    """The ``climate_steps`` recipe generated on a torch device (float64
    FFTs, torch generators seeded with `seed` and `mask_seed`, so values
    differ from the host version): an (nsteps, ny * nx) float32 tensor."""
    import torch

    lat = torch.linspace(-0.5 * math.pi, 0.5 * math.pi, ny, dtype=torch.float64, device=device)
    mu = (250.0 + 40.0 * torch.cos(lat) ** 2).view(ny, 1)
    gen = torch.Generator(device=device)
    gen.manual_seed(mask_seed)
    smooth = _grf_2d_device(ny, nx, gen, -3.0, device)
    thr = torch.kthvalue(smooth.reshape(-1).cpu(), int(0.98 * ny * nx)).values.item()
    land = smooth >= thr
    gen.manual_seed(seed)
    noise = _grf_2d_device(ny, nx, gen, -4.0 / 3.0, device)
    scale = math.sqrt(1.0 - rho * rho)
    out = torch.empty((nsteps, ny * nx), dtype=torch.float32, device=device)
    for t in range(nsteps):
        if t > 0:
            noise = rho * noise + scale * _grf_2d_device(ny, nx, gen, -4.0 / 3.0, device)
        step = mu + 5.0 * noise
        step[land] = 0.0
        out[t] = step.reshape(-1).to(torch.float32)
    return out


_REL_EBS = (1e-2, 1e-3, 1e-4)


def batch_specs(count: int = 4096, seed: int = 7, min_bytes: int = 4096,
                max_bytes: int = 64 << 20):
    """Shapes, seeds and relative error bounds of a batch of uneven fields.

    Sizes are log-uniform between `min_bytes` and `max_bytes` (float32
    elements), dimensionality uniform over 1-D/2-D/3-D with near-square or
    near-cube extents, and each field's relative bound is drawn from
    {1e-2, 1e-3, 1e-4}.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        nbytes = math.exp(rng.uniform(math.log(min_bytes), math.log(max_bytes)))
        n = max(1, int(nbytes // 4))
        dims = int(rng.integers(1, 4))
        if dims == 1:
            shape = (n,)
        elif dims == 2:
            a = max(1, int(round(math.sqrt(n))))
            shape = (a, max(1, n // a))
        else:
            a = max(1, int(round(n ** (1.0 / 3.0))))
            b = max(1, int(round(math.sqrt(n / a))))
            shape = (a, b, max(1, n // (a * b)))
        specs.append({"index": i, "shape": shape, "seed": int(rng.integers(0, 2**31 - 1)),
                      "rel_eb": float(_REL_EBS[int(rng.integers(0, 3))])})
    return specs


def batch_field(spec) -> np.ndarray:
    """Smooth-plus-noise field of a batch spec: per axis three sinusoids with
    periods in [16, 4096] samples, plus Gaussian noise at 1e-3 of the range."""
    rng = np.random.default_rng(spec["seed"])
    shape = spec["shape"]
    field = np.zeros(shape, dtype=np.float64)
    for axis, m in enumerate(shape):
        coord = np.arange(m, dtype=np.float64)
        prof = np.zeros(m)
        for _ in range(3):
            period = math.exp(rng.uniform(math.log(16.0), math.log(4096.0)))
            prof += rng.uniform(0.5, 1.5) * np.sin(2 * math.pi * coord / period
                                                    + rng.uniform(0, 2 * math.pi))
        view = [1] * len(shape)
        view[axis] = m
        field = field + prof.reshape(view)
    r = field.max() - field.min()
    field = field + rng.normal(0.0, 1e-3 * (r if r > 0 else 1.0), size=shape)
    return field.astype(np.float32).ravel()


def batch_field_device(spec, device, out=None):
    """Device-generated field of a batch spec with the same recipe as
    ``batch_field`` (per-axis sums of three sinusoids, periods 16..4096, plus
    Gaussian noise at 1e-3 of the range); the noise comes from a torch
    generator seeded with the spec's seed, so values differ from the host
    version.  Writes into ``out`` (float32, numel = prod(shape)) if given."""
    import torch

    rng = np.random.default_rng(spec["seed"])
    shape = tuple(spec["shape"])
    field = torch.zeros(shape, dtype=torch.float64, device=device)
    for axis, m in enumerate(shape):
        coord = np.arange(m, dtype=np.float64)
        prof = np.zeros(m)
        for _ in range(3):
            period = math.exp(rng.uniform(math.log(16.0), math.log(4096.0)))
            prof += rng.uniform(0.5, 1.5) * np.sin(2 * math.pi * coord / period
                                                    + rng.uniform(0, 2 * math.pi))
        view = [1] * len(shape)
        view[axis] = m
        field += torch.from_numpy(prof).to(device).view(view)
    r = float(field.max().item() - field.min().item())
    gen = torch.Generator(device=device)
    gen.manual_seed(int(spec["seed"]))
    noise = torch.randn(shape, generator=gen, dtype=torch.float32, device=device)
    field += noise.double() * (1e-3 * (r if r > 0 else 1.0))
    flat = field.view(-1)
    if out is None:
        return flat.float()
    out.copy_(flat)
    return out


def batch_arena(specs, device):
    """All fields of a batch generated on `device` into one float32 arena,
    each starting on a 16-byte boundary; returns (arena, [field views])."""
    import torch

    ns = [int(np.prod(sp["shape"])) for sp in specs]
    starts, pos = [], 0
    for n in ns:
        starts.append(pos)
        pos += (n + 3) // 4 * 4
    arena = torch.empty(pos, dtype=torch.float32, device=device)
    views = []
    for sp, n, st in zip(specs, ns, starts):
        x = arena[st:st + n]
        batch_field_device(sp, device, out=x)
        views.append(x)
    return arena, views
