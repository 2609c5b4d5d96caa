"""Five synthetic handheld-scan workloads, each fully determined by a seed.

Every random draw uses ``numpy.random.Generator(PCG64(seed))`` with
``seed = 235680 + index`` (index 2 for the autofocus workload).  All geometry is float64 metres, frequencies are Hz.

Scales follow the paper's own experiments (mm-wave band, 0.25-0.4 m range,
0.1-0.45 m apertures, Sec. V-A and V-C); the measured and full-wave data the
paper used are not available, so these seeded scenes stand in for them.

Index  name            what it is
0      small           1024-position persistent random walk, 32 f, 5 targets,
                       32x32x16 voxels at 2 mm
1      mid             64 serpentine strokes x 256, 64 f, 50 points + a
                       10x10x10 cube, 128x128x64 voxels at 1.5 mm (S=3, Q=4)
2      large           44 strokes + 20 dense walks (65536 positions), 128 f,
                       200 points + a 5000-scatterer slab, 256x256x128 at 1 mm
3      grad            config 0 geometry with a smooth trajectory error
4      autofocus       config 2's scene and echoes (same seed) with a smooth
                       trajectory error on the positions handed to the imager
5      paper_sim       the shape of the paper's point-target simulation: a
                       101-element linear array swept over 101 positions
                       (0.45 m), depth and angle fluctuations, 24 f 12-15 GHz,
                       3x3x3 points at 0.175 m spacing around (0, 0, 0.4 m),
                       101x101x51 voxels over 0.5 m^3
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C0 = 299792458.0  # speed of light in vacuum, m/s (the paper leaves c unstated)
SEED_BASE = 235680
CONFIG_NAMES = ("small", "mid", "large", "grad", "autofocus", "paper_sim")


@dataclasses.dataclass
class Workload:
    name: str
    positions: np.ndarray          # (n_pos, 3) float64, true antenna positions
    freqs_hz: np.ndarray           # (n_f,) float64
    grid_origin: np.ndarray        # (3,) centre of voxel (0,0,0)
    grid_pitch: np.ndarray         # (3,)
    grid_dims: tuple               # (nx, ny, nz); voxel (ix,iy,iz) = origin + i*pitch
    target_pos: np.ndarray         # (n_t, 3)
    target_amp: np.ndarray         # (n_t,) complex128
    echoes: np.ndarray | None      # (n_pos, n_f) complex128 (None until synthesised)
    stages: int                    # suggested factorisation stages
    merge_factor: int              # 4 = one x and one y bisection per stage
    imager_positions: np.ndarray | None = None   # positions handed to the imager
    noise_var: float = 0.0
    seed: int = 0

    @property
    def n_pos(self):
        return self.positions.shape[0]

    @property
    def n_f(self):
        return self.freqs_hz.shape[0]

    @property
    def n_vox(self):
        return int(np.prod(self.grid_dims))


def voxel_centres(origin, pitch, dims):
    """(nx*ny*nz, 3) voxel centres, z fastest (C order over (ix, iy, iz))."""
    ax = [origin[a] + pitch[a] * np.arange(dims[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def grid_box(origin, pitch, dims):
    lo = np.asarray(origin, float)
    hi = lo + np.asarray(pitch, float) * (np.asarray(dims) - 1)
    return lo, hi


def _centred_grid(centre, pitch, dims):
    centre = np.asarray(centre, float)
    pitch = np.asarray([pitch] * 3, float)
    origin = centre - pitch * (np.asarray(dims) - 1) / 2.0
    return origin, pitch, tuple(int(d) for d in dims)


def _persistent_walk(rng, n, step, half, start=None, turn_sigma=0.3):
    """2-D walk with heading increments N(0, turn_sigma), reflecting at |x|,|y|<=half."""
    xy = np.empty((n, 2))
    p = np.array(start if start is not None else rng.uniform(-half, half, 2), float)
    th = rng.uniform(0, 2 * math.pi)
    dth = rng.normal(0.0, turn_sigma, n)
    for i in range(n):
        xy[i] = p
        th += dth[i]
        p = p + step * np.array([math.cos(th), math.sin(th)])
        for a in range(2):
            if p[a] > half:
                p[a] = 2 * half - p[a]
                th = (math.pi - th) if a == 0 else -th
            elif p[a] < -half:
                p[a] = -2 * half - p[a]
                th = (math.pi - th) if a == 0 else -th
    return xy


def _smooth(rng, n, amp):
    """Sum of 3 sinusoids over the index with random frequency (0.5-3 cycles per
    scan) and phase, scaled to max |.| = amp."""
    t = np.arange(n) / max(n - 1, 1)
    e = sum(rng.uniform(0.3, 1.0) * np.sin(2 * math.pi * rng.uniform(0.5, 3.0) * t
                                           + rng.uniform(0, 2 * math.pi)) for _ in range(3))
    return e * (amp / max(np.abs(e).max(), 1e-30))


def _linear_array_scan(rng, n_el, n_scan, extent, depth, roll_deg, yaw_deg, lat_sigma):
    """A linear array of n_el elements (along y) swept along x over n_scan
    positions, with smooth lateral, depth, roll and yaw fluctuations of the
    handheld array (scan-major order)."""
    xs = -extent / 2 + extent * np.arange(n_scan) / (n_scan - 1) + rng.normal(0, lat_sigma, n_scan)
    yc = _smooth(rng, n_scan, 5e-3)
    zc = _smooth(rng, n_scan, depth)
    roll = np.radians(_smooth(rng, n_scan, roll_deg))
    yaw = np.radians(_smooth(rng, n_scan, yaw_deg))
    s = -extent / 2 + extent * np.arange(n_el) / (n_el - 1)
    pos = np.empty((n_scan, n_el, 3))
    for j in range(n_scan):
        pos[j, :, 0] = xs[j] - s * math.sin(yaw[j])
        pos[j, :, 1] = yc[j] + s * math.cos(yaw[j]) * math.cos(roll[j])
        pos[j, :, 2] = zc[j] + s * math.sin(roll[j])
    return pos.reshape(-1, 3)


def _strokes(rng, n_strokes, per_stroke, half, lat_sigma):
    rows = []
    for j in range(n_strokes):
        y0 = -half + (j + 0.5) * (2 * half) / n_strokes
        x = np.linspace(-half, half, per_stroke)
        if j % 2:
            x = x[::-1]
        y = y0 + rng.normal(0.0, lat_sigma, per_stroke)
        rows.append(np.stack([x, y], axis=1))
    return np.concatenate(rows, axis=0)


def synth_echoes(positions, freqs_hz, target_pos, target_amp, chunk=1024, device=None):
    """Born-model echoes s(p', k) = sum_t a_t exp(-j 2 k |p_t - p'|) (eq. 1), float64.

    ``device`` (a torch device string, default the CPU) only chooses where the
    float64 sums run: the formula and the seeded draws are the same, and the
    results agree with the CPU ones to float64 rounding (~1e-15 relative)."""
    import torch

    dev = torch.device(device or "cpu")
    k = torch.as_tensor(2.0 * math.pi * np.asarray(freqs_hz, float) / C0, dtype=torch.float64)
    tp = torch.as_tensor(np.asarray(target_pos, float)).to(dev)
    ta = torch.as_tensor(np.asarray(target_amp, np.complex128)).to(dev)
    pos = np.asarray(positions, float)
    out = np.empty((pos.shape[0], k.shape[0]), np.complex128)
    if dev.type != "cpu":
        chunk = max(chunk, 4096)
    for c0 in range(0, pos.shape[0], chunk):
        p = torch.as_tensor(pos[c0:c0 + chunk]).to(dev)
        if dev.type == "cpu":
            R = torch.cdist(p, tp, compute_mode="donot_use_mm_for_euclid_dist")   # (n, n_t)
        else:
            # written out: float64 cdist on the GPU has returned wrong distances
            # for rows past ~870 of a 4096 x 5200 problem on this ROCm build
            R = torch.sqrt(((p[:, None, :] - tp[None, :, :]) ** 2).sum(-1))
        acc = torch.empty((p.shape[0], k.shape[0]), dtype=torch.complex128, device=dev)
        for f in range(k.shape[0]):
            ph = (-2.0 * float(k[f])) * R
            acc[:, f] = torch.polar(torch.ones_like(ph), ph) @ ta
        out[c0:c0 + chunk] = acc.cpu().numpy()
    return out


def trajectory_error(rng, n_pos, max_amp=3e-3):
    """Smooth per-axis error: sum of 3 sinusoids, max |e| per axis ~ U[0, max_amp]."""
    t = np.arange(n_pos, dtype=float)
    e = np.zeros((n_pos, 3))
    for a in range(3):
        nu = rng.uniform(0.5, 4.0, 3)
        phi = rng.uniform(0.0, 2 * math.pi, 3)
        amp = rng.uniform(0.2, 1.0, 3)
        ea = (amp[None, :] * np.sin(2 * math.pi * nu[None, :] * t[:, None] / n_pos
                                    + phi[None, :])).sum(1)
        target = rng.uniform(0.0, max_amp)
        e[:, a] = ea * (target / max(np.abs(ea).max(), 1e-30))
    return e


def _uniform_in_box(rng, n, lo, hi):
    return rng.uniform(lo, hi, (n, 3))


def make_config(index, synth=True, seed=None, synth_device=None):
    """Build workload ``index`` (0..4).  ``synth=False`` skips echo synthesis;
    ``synth_device`` runs the float64 echo sums on a torch device (see
    ``synth_echoes``)."""
    # the autofocus workload images the large scene: same seed, then a
    # trajectory error drawn after the scene
    seed = SEED_BASE + (2 if index == 4 else index) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    name = CONFIG_NAMES[index]
    noise_var = 0.0
    imager = None
    if index in (0, 3):
        xy = _persistent_walk(rng, 1024, 1e-3, 0.06)
        z = rng.normal(0.0, 1e-3, 1024)
        pos = np.column_stack([xy, z])
        freqs = np.linspace(26e9, 40e9, 32)
        origin, pitch, dims = _centred_grid((0.0, 0.0, 0.25), 2e-3, (32, 32, 16))
        tpos = rng.uniform([-0.05, -0.05, 0.225], [0.05, 0.05, 0.275], (5, 3))
        tamp = np.ones(5, np.complex128)
        stages, q = 2, 4
    elif index == 1:
        xy = _strokes(rng, 64, 256, 0.15, 2e-3)
        z = rng.normal(0.0, 1e-3, xy.shape[0])
        pos = np.column_stack([xy, z])
        freqs = np.linspace(24e9, 40e9, 64)
        origin, pitch, dims = _centred_grid((0.0, 0.0, 0.3), 1.5e-3, (128, 128, 64))
        lo, hi = grid_box(origin, pitch, dims)
        pts = _uniform_in_box(rng, 50, lo + 0.01, hi - 0.01)
        g = (np.arange(10) - 4.5) * 1e-3
        cube = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + [0, 0, 0.3]
        tpos = np.concatenate([pts, cube])
        tamp = np.ones(tpos.shape[0], np.complex128)
        stages, q = 3, 4
    elif index in (2, 4):
        a = _strokes(rng, 44, 1024, 0.15, 2e-3)
        walks = [_persistent_walk(rng, 1024, 1e-3, 0.04) for _ in range(20)]
        xy = np.concatenate([a] + walks)
        z = rng.normal(0.0, 1e-3, xy.shape[0])
        pos = np.column_stack([xy, z])
        freqs = np.linspace(24e9, 40e9, 128)
        origin, pitch, dims = _centred_grid((0.0, 0.0, 0.3), 1e-3, (256, 256, 128))
        lo, hi = grid_box(origin, pitch, dims)
        pts = _uniform_in_box(rng, 200, lo + 0.01, hi - 0.01)
        slab = rng.uniform([-0.1, -0.1, 0.328], [0.1, 0.1, 0.332], (5000, 3))
        tpos = np.concatenate([pts, slab])
        samp = (rng.standard_normal(5000) + 1j * rng.standard_normal(5000)) / math.sqrt(2)
        tamp = np.concatenate([np.ones(200, np.complex128), samp])
        stages, q = 3, 4
    elif index == 5:
        # the shape of the paper's first point-target simulation (Sec. V-A):
        # 101 elements x 101 scan positions over ~0.45 m, depth within 8 cm
        pos = _linear_array_scan(rng, 101, 101, 0.45, 0.03, 5.0, 3.0, 1e-3)
        freqs = np.linspace(12e9, 15e9, 24)
        origin, pitch, dims = _centred_grid((0.0, 0.0, 0.4), 5e-3, (101, 101, 51))
        pitch = np.array([5e-3, 5e-3, 10e-3])
        origin = np.array([0.0, 0.0, 0.4]) - pitch * (np.asarray(dims) - 1) / 2.0
        g = np.array([-0.175, 0.0, 0.175])
        tpos = np.stack(np.meshgrid(g, g, g + 0.4, indexing="ij"), -1).reshape(-1, 3)
        tamp = np.ones(27, np.complex128)
        stages, q = 3, 4
    else:
        raise ValueError(f"unknown config {index}")
    if index in (3, 4):
        imager = pos + trajectory_error(rng, pos.shape[0])
    w = Workload(name=name, positions=pos, freqs_hz=freqs, grid_origin=origin,
                 grid_pitch=pitch, grid_dims=dims, target_pos=tpos, target_amp=tamp,
                 echoes=None, stages=stages, merge_factor=q, imager_positions=imager,
                 seed=seed)
    if synth:
        s = synth_echoes(pos, freqs, tpos, tamp, device=synth_device)
        if index in (0, 3):
            # 30 dB SNR: per-sample variance = mean |s|^2 / 10^3, circular Gaussian
            noise_var = float(np.mean(np.abs(s) ** 2)) / 1e3
            s = s + math.sqrt(noise_var / 2) * (rng.standard_normal(s.shape)
                                                + 1j * rng.standard_normal(s.shape))
        w.echoes = s
        w.noise_var = noise_var
    return w
