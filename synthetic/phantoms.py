"""Random tubular vessel phantoms and seeded random arrays (FP64, host only).

Vessel recipe (stand-in for the paper's vasculature phantoms, Sec. 5.1):
per vessel an amplitude U[0.5, 1] and a radius U[r_min, r_max] (voxels); a
start point uniform in the non-PML interior shrunk by r_max + 2 voxels; four
segments with directions uniform on the sphere and lengths U[0.25, 0.5] times
the interior width, each end point clamped to the shrunk interior. A voxel
takes the maximum over vessels of amplitude * [distance(voxel centre,
polyline) <= radius]. The volume is then smoothed by a separable Gaussian
(sigma = 0.7 voxel, 7 taps, normalised, zero outside) and clipped at 0, like
the pre-smoothing the paper applies before simulating data (Sec. 5.2).
"""

import numpy as np


def _interior(shape, pml):
    nz, ny, nx = shape
    lo = np.array([1.0, pml, pml])                       # z starts after the sensor layer
    hi = np.array([nz - 2 * pml - 1.0, ny - pml - 1.0, nx - pml - 1.0])
    return lo, hi


def _segment_dist(pts, a, b):
    ab = b - a
    denom = float(ab @ ab)
    t = np.zeros(len(pts)) if denom == 0.0 else np.clip(((pts - a) @ ab) / denom, 0.0, 1.0)
    proj = a + t[:, None] * ab
    return np.sqrt(((pts - proj) ** 2).sum(axis=1))


def _smooth(vol, sigma=0.7, taps=7):
    h = taps // 2
    x = np.arange(-h, h + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    w /= w.sum()
    out = vol
    for axis in range(3):
        padw = [(0, 0)] * 3
        padw[axis] = (h, h)
        p = np.pad(out, padw)
        acc = np.zeros_like(out)
        n = out.shape[axis]
        for i, wi in enumerate(w):
            sl = [slice(None)] * 3
            sl[axis] = slice(i, i + n)
            acc += wi * p[tuple(sl)]
        out = acc
    return out


def _draw_vessels(rng, shape, pml, n_vessels, r_min, r_max):
    lo, hi = _interior(shape, pml)
    lo_s = lo + (r_max + 2.0)
    hi_s = hi - (r_max + 2.0)
    hi_s = np.maximum(hi_s, lo_s)
    width = float(np.min(hi - lo))
    vessels = []
    for _ in range(n_vessels):
        amp = rng.uniform(0.5, 1.0)
        rad = rng.uniform(r_min, r_max)
        pts = [lo_s + rng.uniform(size=3) * (hi_s - lo_s)]
        for _ in range(4):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            length = rng.uniform(0.25, 0.5) * width
            pts.append(np.clip(pts[-1] + length * d, lo_s, hi_s))
        vessels.append((amp, rad, pts))
    return vessels


def _rasterize(shape, vessels, offset=(0.0, 0.0, 0.0), amps=None):
    vol = np.zeros(shape)
    zz, yy, xx = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    off = np.asarray(offset, dtype=np.float64)
    for v, (amp, rad, pts) in enumerate(vessels):
        amp = amp if amps is None else amps[v]
        for a, b in zip(pts[:-1], pts[1:]):
            a, b = a + off, b + off
            bl = np.floor(np.minimum(a, b) - rad - 1).astype(int)
            bh = np.ceil(np.maximum(a, b) + rad + 1).astype(int) + 1
            bl = np.maximum(bl, 0)
            bh = np.minimum(bh, np.array(shape))
            if np.any(bh <= bl):
                continue
            sl = tuple(slice(l, h) for l, h in zip(bl, bh))
            grid_pts = np.stack([zz[sl].ravel(), yy[sl].ravel(), xx[sl].ravel()], axis=1)
            inside = (_segment_dist(grid_pts, a, b) <= rad).reshape(zz[sl].shape)
            vol[sl] = np.maximum(vol[sl], amp * inside)
    return vol


def vessel_phantom(shape, pml, n_vessels, r_min, r_max, seed, smooth=True):
    """[nz][ny][nx] nonnegative FP64 phantom."""
    rng = np.random.default_rng(seed)
    vol = _rasterize(shape, _draw_vessels(rng, shape, pml, n_vessels, r_min, r_max))
    if smooth:
        vol = _smooth(vol)
    return np.maximum(vol, 0.0)


def moving_vessel_frames(shape, pml, n_frames, n_vessels, r_min, r_max, seed, shift=1.0, pulse=0.1, period=8):
    """Frames of a moving vessel phantom (a dynamic scan): the vessels of
    vessel_phantom(shape, pml, n_vessels, r_min, r_max, seed) translated rigidly
    by `shift` voxels per frame along a seeded direction parallel to the sensor
    plane (reversing at the interior's edge), each vessel's amplitude pulsating
    as 1 + pulse * sin(2 pi t / period + phase_v) with a seeded phase. Voxels
    closer than 3 to the PML or to the sensor layer are cleared before the
    smoothing, so every frame stays inside the interior. Returns a list of
    [nz][ny][nx] FP64 volumes."""
    rng = np.random.default_rng(seed)
    vessels = _draw_vessels(rng, shape, pml, n_vessels, r_min, r_max)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_vessels)
    ang = rng.uniform(0.0, 2.0 * np.pi)
    direction = np.array([0.0, np.sin(ang), np.cos(ang)])
    lo, hi = _interior(shape, pml)
    keep = np.zeros(shape, dtype=bool)
    keep[tuple(slice(int(l) + 3, int(h) - 2) for l, h in zip(lo, hi))] = True
    span = 8.0 * shift
    frames = []
    for t in range(n_frames):
        s = (t * shift) % (2.0 * span) if span > 0 else 0.0
        s = s if s <= span else 2.0 * span - s   # back and forth over `span` voxels
        amps = [amp * (1.0 + pulse * np.sin(2.0 * np.pi * t / period + phase[v]))
                for v, (amp, _, _) in enumerate(vessels)]
        vol = _rasterize(shape, vessels, s * direction, amps) * keep
        frames.append(np.maximum(_smooth(vol), 0.0))
    return frames


def gaussian_volume(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def gaussian_data(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def gaussian_blob(shape, centre, sigma):
    """exp(-r^2 / (2 sigma^2)) around `centre` = (z, y, x) in voxel units."""
    zz, yy, xx = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    r2 = (zz - centre[0]) ** 2 + (yy - centre[1]) ** 2 + (xx - centre[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


def lognormal_weights(shape, sigma, seed):
    """w = exp(sigma X), X ~ N(0, 1) seeded (the paper's model of a spatially varying
    sensor sensitivity, sigma = 0.2, and of the noise level per sensor, sigma = 0.1)."""
    return np.exp(sigma * gaussian_data(shape, seed))


def sound_speed_field(p0, c0, rel=0.05, seed=0, smooth=3.0):
    """The perturbed sound speed of the paper's no-inverse-crime data (Sec. 5.3): a smooth
    normalised Gaussian random field plus the normalised initial pressure, centred and
    scaled so that its mean is 0 and its largest magnitude rel * c0, added to c0."""
    from scipy.ndimage import gaussian_filter
    p0 = np.asarray(p0, dtype=np.float64)
    g = gaussian_filter(gaussian_data(p0.shape, seed), smooth)
    g /= np.abs(g).max()
    q = p0 / p0.max() if p0.max() > 0 else np.zeros_like(p0)
    t = g + q
    t -= t.mean()
    return c0 + rel * c0 * t / np.abs(t).max()
