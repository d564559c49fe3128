"""Seeded synthetic inputs for the HVOX transforms.

This module only *generates* coordinates and data vectors; it holds none of the
transform's arithmetic, so the CPU oracle (tests) and the GPU library can both
be fed from it without sharing any part of the method.

Geometry follows the paper's problem statement (Sect. 2, Eqs. 2-3): baselines
``p_k`` are uvw coordinates in wavelengths and sky points ``r_n`` are unit
vectors of an arbitrary spherical mesh.  The paper's own datasets (SKA-Low
layout, LOFAR measurement sets, Sect. 5 and Table 2) are not available, so the
generators below stand in for them with layouts of the same kind:

* a Fibonacci-lattice spherical cap (an equal-area mesh, any pixel count);
* uv uniform in a disk with small w (a compact array);
* earth-rotation synthesis of an antenna layout (standard interferometer
  geometry: ENU -> equatorial -> uvw by hour angle and declination).

All random draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = (1.0 + 5.0 ** 0.5) / 2.0


# --------------------------------------------------------------------------
# sky meshes
# --------------------------------------------------------------------------
def fibonacci_cap(n: int, half_angle_deg: float) -> np.ndarray:
    """``n`` unit vectors of a Fibonacci lattice on the cap of the given
    half-angle around +z.  Deterministic; equal-area cells."""
    if n <= 0:
        return np.zeros((0, 3))
    i = np.arange(n, dtype=np.float64)
    c0 = math.cos(math.radians(half_angle_deg))
    z = 1.0 - (1.0 - c0) * (i + 0.5) / n
    phi = 2.0 * np.pi * np.mod(i / GOLDEN, 1.0)
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def random_cap(n: int, half_angle_deg: float, rng: np.random.Generator) -> np.ndarray:
    """``n`` unit vectors drawn uniformly (in area) on a cap around +z."""
    c0 = math.cos(math.radians(half_angle_deg))
    z = 1.0 - (1.0 - c0) * rng.random(n)
    phi = 2.0 * np.pi * rng.random(n)
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def dcos_grid(npix_side: int, fov_deg: float) -> np.ndarray:
    """Unit vectors of a square direction-cosine (l, m) grid around +z, the
    mesh used by planar gridders (Sect. 2.1)."""
    half = math.sin(math.radians(fov_deg) / 2.0)
    g = np.linspace(-half, half, npix_side)
    l, m = np.meshgrid(g, g, indexing="xy")
    l = l.ravel(); m = m.ravel()
    n = np.sqrt(np.maximum(0.0, 1.0 - l * l - m * m))
    return np.stack([l, m, n], axis=1)


# --------------------------------------------------------------------------
# baselines
# --------------------------------------------------------------------------
def uvw_disk(m: int, radius: float, w_half: float, rng: np.random.Generator) -> np.ndarray:
    """u, v uniform in a disk of ``radius`` wavelengths, w uniform in
    [-w_half, w_half]."""
    r = radius * np.sqrt(rng.random(m))
    a = 2.0 * np.pi * rng.random(m)
    w = rng.uniform(-w_half, w_half, m)
    return np.stack([r * np.cos(a), r * np.sin(a), w], axis=1)


def earth_rotation_uvw(enu: np.ndarray, lat_deg: float, dec_deg: float,
                       hour_angles_rad: np.ndarray, wavelengths_m) -> np.ndarray:
    """uvw (in wavelengths) of every antenna pair p < q, for every hour angle
    and wavelength.  Order: [wavelength][hour angle][pair].

    Antenna positions ``enu`` are local east/north/up metres.  The baseline is
    rotated into the equatorial frame at latitude ``lat_deg`` and projected on
    the (u, v, w) frame of a source at declination ``dec_deg``."""
    enu = np.asarray(enu, dtype=np.float64)
    na = enu.shape[0]
    p, q = np.triu_indices(na, k=1)
    b = enu[q] - enu[p]                                   # (nb, 3) E, N, U
    lat = math.radians(lat_deg)
    sl, cl = math.sin(lat), math.cos(lat)
    X = -sl * b[:, 1] + cl * b[:, 2]
    Y = b[:, 0]
    Z = cl * b[:, 1] + sl * b[:, 2]
    dec = math.radians(dec_deg)
    sd, cd = math.sin(dec), math.cos(dec)
    H = np.asarray(hour_angles_rad, dtype=np.float64)[:, None]
    sh, ch = np.sin(H), np.cos(H)
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    uvw_m = np.stack([u, v, w], axis=-1).reshape(-1, 3)    # (T*nb, 3) metres
    lams = np.atleast_1d(np.asarray(wavelengths_m, dtype=np.float64))
    return np.concatenate([uvw_m / lam for lam in lams], axis=0)


def gaussian_layout(n_ant: int, sigma_m: float, rng: np.random.Generator) -> np.ndarray:
    e = rng.normal(0.0, sigma_m, n_ant)
    n = rng.normal(0.0, sigma_m, n_ant)
    return np.stack([e, n, np.zeros(n_ant)], axis=1)


def log_radial_layout(n_st: int, r_min_m: float, r_max_m: float,
                      rng: np.random.Generator) -> np.ndarray:
    r = 10.0 ** rng.uniform(math.log10(r_min_m), math.log10(r_max_m), n_st)
    a = 2.0 * np.pi * rng.random(n_st)
    return np.stack([r * np.cos(a), r * np.sin(a), np.zeros(n_st)], axis=1)


# --------------------------------------------------------------------------
# data vectors
# --------------------------------------------------------------------------
def real_intensities(ntrans: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Sky intensities uniform in [0, 1] as a complex array (imaginary 0)."""
    return rng.random((ntrans, n)).astype(np.complex128)


def complex_normal(ntrans: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Circular complex normal CN(0, 1) entries."""
    s = math.sqrt(0.5)
    return s * (rng.standard_normal((ntrans, n)) + 1j * rng.standard_normal((ntrans, n)))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    uvw: np.ndarray            # (M, 3) float64, wavelengths
    xyz: np.ndarray            # (N, 3) float64, unit vectors
    sky: np.ndarray            # (ntrans, N) complex128
    vis: np.ndarray            # (ntrans, M) complex128
    info: dict = field(default_factory=dict)

    @property
    def n_vis(self) -> int:
        return self.uvw.shape[0]

    @property
    def n_pix(self) -> int:
        return self.xyz.shape[0]


def compact_disk(seed: int = 1, n_vis: int = 2000, n_pix: int = 3072,
                 radius: float = 1000.0, w_half: float = 50.0,
                 cap_deg: float = 5.0, ntrans: int = 1) -> Workload:
    """Small compact-array case: 2,000 visibilities with u, v uniform in a disk
    of radius 1,000 wavelengths and w in [-50, 50]; a 3,072-point Fibonacci cap
    of half-angle 5 degrees; real intensities in [0, 1]."""
    rng = np.random.default_rng(seed)
    uvw = uvw_disk(n_vis, radius, w_half, rng)
    xyz = fibonacci_cap(n_pix, cap_deg)
    sky = real_intensities(ntrans, n_pix, rng)
    vis = complex_normal(ntrans, n_vis, rng)
    return Workload("compact-disk-2k-vis-3k-pix", uvw, xyz, sky, vis,
                    dict(seed=seed, radius=radius, w_half=w_half, cap_deg=cap_deg))


def ska_like_uvw(seed: int = 2, n_ant: int = 200, sigma_m: float = 5000.0,
                 n_times: int = 50, ha_deg: float = 30.0, lat_deg: float = -30.0,
                 dec_deg: float = -30.0, wavelength_m: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    enu = gaussian_layout(n_ant, sigma_m, rng)
    H = np.radians(np.linspace(-ha_deg, ha_deg, n_times))
    return earth_rotation_uvw(enu, lat_deg, dec_deg, H, [wavelength_m])


def ska_like(seed: int = 2, n_pix: int = 1_000_000, cap_deg: float = 10.0,
             ntrans: int = 1, n_ant: int = 200, n_times: int = 50) -> Workload:
    """SKA-like: 200 antennas with Gaussian E/N positions (sigma 5 km),
    earth-rotation synthesis over 50 hour angles in [-2h, +2h] at declination
    -30 deg (latitude -30 deg), one channel at 1 m: 995,000 visibilities.
    1M-point Fibonacci cap of half-angle 10 deg.  Intensities U[0,1],
    visibilities CN(0,1)."""
    uvw = ska_like_uvw(seed, n_ant=n_ant, n_times=n_times)
    xyz = fibonacci_cap(n_pix, cap_deg)
    rng = np.random.default_rng(seed + 1000)
    sky = real_intensities(ntrans, n_pix, rng)
    vis = complex_normal(ntrans, uvw.shape[0], rng)
    return Workload(f"ska-like-{uvw.shape[0]}-vis-{n_pix}-pix", uvw, xyz, sky, vis,
                    dict(seed=seed, n_ant=n_ant, n_times=n_times, cap_deg=cap_deg))


def lofar_like_uvw(seed: int = 3, n_st: int = 60, r_min_m: float = 100.0,
                   r_max_m: float = 100e3, n_chan: int = 4, target_vis: int = 5_000_000,
                   w_max: float = 2e4, lat_deg: float = 52.91,
                   dec_deg: float = 52.91) -> np.ndarray:
    rng = np.random.default_rng(seed)
    enu = log_radial_layout(n_st, r_min_m, r_max_m, rng)
    lams = np.linspace(2.0, 3.0, n_chan)
    nb = n_st * (n_st - 1) // 2
    n_times = int(math.ceil(target_vis / (nb * n_chan)))

    def max_w(h0):
        H = np.linspace(-h0, h0, n_times)
        return np.abs(earth_rotation_uvw(enu, lat_deg, dec_deg, H, [lams.min()])[:, 2]).max()

    lo, hi = 0.0, math.pi
    if max_w(hi) <= w_max:
        lo = hi
    else:
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if max_w(mid) > w_max:
                hi = mid
            else:
                lo = mid
    H = np.linspace(-lo, lo, n_times)
    return earth_rotation_uvw(enu, lat_deg, dec_deg, H, lams)


def lofar_like(seed: int = 3, n_pix: int = 4_000_000, cap_deg: float = 60.0,
               ntrans: int = 1) -> Workload:
    """LOFAR-like wide field: 60 stations with log-radial layout 100 m..100 km,
    4 channels at 2-3 m, hour-angle span set so that max |w| = 2e4
    wavelengths: 5,005,560 visibilities.  4M-point cap of half-angle 60 deg."""
    uvw = lofar_like_uvw(seed)
    xyz = fibonacci_cap(n_pix, cap_deg)
    rng = np.random.default_rng(seed + 1000)
    sky = real_intensities(ntrans, n_pix, rng)
    vis = complex_normal(ntrans, uvw.shape[0], rng)
    return Workload(f"lofar-like-{uvw.shape[0]}-vis-{n_pix}-pix", uvw, xyz, sky, vis,
                    dict(seed=seed, cap_deg=cap_deg))


# Telescope-radius ladder of the paper's runtime experiments (Sect. 5.1 and
# its table of telescope scales): radius in km -> (visibility count, pixels
# per side of the dense DCOS image).  The image side reproduces the table's
# pixel counts exactly (80^2 = 6,400 ... 13,500^2 = 182.25M).
DENSE_LADDER = {0.1: (273, 80), 0.3: (13_000, 160), 1.0: (95_000, 360), 3.0: (148_000, 900),
                10.0: (238_000, 3200), 30.0: (341_000, 8640), 100.0: (394_000, 13_500)}


def ladder_uvw(radius_km: float, rng: np.random.Generator, lat_deg: float = -26.82, dec_deg: float = -45.0,
               wavelength_m: float = 2.0):
    """Baselines of a telescope-radius rung: stations at log-radial distances
    between 15 m and the radius, as many as three snapshots (hour angles
    -4 h, 0, +4 h) need for the rung's visibility count."""
    n_vis_target, _ = DENSE_LADDER[float(radius_km)]
    n_st = max(2, int(round(0.5 + math.sqrt(0.25 + 2.0 * n_vis_target / 3.0))))
    enu = log_radial_layout(n_st, 15.0, radius_km * 1e3, rng)
    H = np.radians(np.linspace(-60.0, 60.0, 3))          # -4 h, 0, +4 h
    return earth_rotation_uvw(enu, lat_deg, dec_deg, H, [wavelength_m]), n_st


def dense_dcos(radius_km: float = 3.0, seed: int = 5, ntrans: int = 1, fov_deg: float = 30.0,
               lat_deg: float = -26.82, dec_deg: float = -45.0, wavelength_m: float = 2.0) -> Workload:
    """Dense-mesh case shaped after the paper's runtime ladder (default
    parameters of its benchmarks: an SKA-Low-like array at 150 MHz, one
    channel, three equi-spaced time intervals over 8 hours, declination -45 deg,
    a 30-degree DCOS image).  The SKA-Low station table is not available: the
    stations sit at log-radial distances between 15 m and the telescope radius
    (a dense core, sparse outskirts), their count chosen so that three
    snapshots give the ladder's visibility count.  The image is the ladder's
    square DCOS grid around the phase centre; intensities U[0,1]."""
    n_vis_target, n_side = DENSE_LADDER[float(radius_km)]
    rng = np.random.default_rng(seed)
    uvw, n_st = ladder_uvw(radius_km, rng, lat_deg, dec_deg, wavelength_m)
    xyz = dcos_grid(n_side, fov_deg)
    sky = real_intensities(ntrans, xyz.shape[0], rng)
    vis = complex_normal(ntrans, uvw.shape[0], rng)
    return Workload(f"dense-dcos-{radius_km:g}km-{uvw.shape[0]}-vis-{xyz.shape[0]}-pix", uvw, xyz, sky, vis,
                    dict(seed=seed, radius_km=radius_km, n_stations=n_st, n_side=n_side, fov_deg=fov_deg))


def sparse_dcos(radius_km: float = 10.0, seed: int = 7, n_regions: int = 5, side: int = 10, ntrans: int = 1,
                fov_deg: float = 30.0) -> Workload:
    """Sparse-mesh case shaped after the paper's sparse-sky runtime experiment:
    the visibilities of a telescope-radius rung (as ``dense_dcos``) and only
    500 pixels of interest -- ``n_regions`` small contiguous patches of
    ``side`` x ``side`` pixels of that rung's 30-degree DCOS grid around
    randomly placed calibrators (the regions are not contiguous with each
    other), as in direction-dependent calibration.  Intensities U[0,1]."""
    n_vis_target, n_side = DENSE_LADDER[float(radius_km)]
    uvw, _ = ladder_uvw(radius_km, np.random.default_rng(5))     # the dense rung's baselines
    rng = np.random.default_rng(seed)
    # patch corners on the rung's pixel grid, kept inside the image and apart
    corners = []
    while len(corners) < n_regions:
        c = rng.integers(0, n_side - side, 2)
        if all(max(abs(int(c[0]) - a), abs(int(c[1]) - b)) >= side for a, b in corners):
            corners.append((int(c[0]), int(c[1])))
    # pixels (row, col) of the patches on the rung's grid (dcos_grid: col along l, row along m)
    half = math.sin(math.radians(fov_deg) / 2.0)
    g = np.linspace(-half, half, n_side)
    rows = np.concatenate([np.repeat(r0 + np.arange(side), side) for r0, _ in corners])
    cols = np.concatenate([np.tile(c0 + np.arange(side), side) for _, c0 in corners])
    l, m = g[cols], g[rows]
    xyz = np.stack([l, m, np.sqrt(np.maximum(0.0, 1.0 - l * l - m * m))], axis=1)
    sky = real_intensities(ntrans, xyz.shape[0], rng)
    vis = complex_normal(ntrans, uvw.shape[0], rng)
    return Workload(f"sparse-dcos-{radius_km:g}km-{uvw.shape[0]}-vis-{xyz.shape[0]}-pix", uvw, xyz, sky, vis,
                    dict(seed=seed, radius_km=radius_km, n_regions=n_regions, side=side, n_side=n_side,
                         corners=corners, fov_deg=fov_deg))


@dataclass
class Request:
    rid: int
    arrival_s: float
    direction: str             # "synthesis" (sky -> vis) or "analysis" (vis -> sky)
    layout: str                # "ska" or "lofar"
    uvw: np.ndarray
    xyz: np.ndarray
    data: np.ndarray           # (1, n_in) complex128: sky for synthesis, vis for analysis


def serving_requests(seed: int = 4, n_req: int = 64, mean_gap_s: float = 0.010,
                     log10_min: float = 4.0, log10_max: float = 6.0,
                     layouts: dict | None = None) -> list[Request]:
    """Poisson-arriving requests of uneven size: each a random synthesis or
    analysis job with log-uniform visibility and pixel counts, on subsampled
    SKA-like or LOFAR-like baselines and a Fibonacci cap (10 deg for SKA-like,
    60 deg for LOFAR-like).  ``layouts`` may pass precomputed uvw arrays."""
    rng = np.random.default_rng(seed)
    if layouts is None:
        layouts = {"ska": ska_like_uvw(), "lofar": lofar_like_uvw()}
    caps = {"ska": 10.0, "lofar": 60.0}
    t = 0.0
    out = []
    for rid in range(n_req):
        t += rng.exponential(mean_gap_s)
        direction = "synthesis" if rng.random() < 0.5 else "analysis"
        lay = "ska" if rng.random() < 0.5 else "lofar"
        nv = int(10.0 ** rng.uniform(log10_min, log10_max))
        npx = int(10.0 ** rng.uniform(log10_min, log10_max))
        base = layouts[lay]
        nv = min(nv, base.shape[0])
        idx = np.sort(rng.choice(base.shape[0], size=nv, replace=False))
        uvw = base[idx]
        xyz = fibonacci_cap(npx, caps[lay])
        if direction == "synthesis":
            data = real_intensities(1, npx, rng)
        else:
            data = complex_normal(1, nv, rng)
        out.append(Request(rid, t, direction, lay, uvw, xyz, data))
    return out


def snapshot_beams(n_vis: int, n_times: int, xyz: np.ndarray, fwhm_deg: float = 8.0,
                   drift_deg: float = 3.0) -> tuple[np.ndarray, np.ndarray]:
    """Direction-dependent gains of a time-variable primary beam in the
    separable form A_k(r_n) = sum_t a[t, k] b[t, n]: visibility k belongs to
    snapshot t = k // (n_vis / n_times) (the [hour angle][pair] order of
    earth_rotation_uvw) and sees b[t], a Gaussian beam of the given FWHM whose
    pointing drifts linearly by drift_deg in x across the observation.
    a: (n_times, n_vis) 0/1, b: (n_times, n_pix) real, both complex128."""
    per = n_vis // n_times
    if per * n_times != n_vis:
        raise ValueError("n_vis must be a multiple of n_times")
    a = np.zeros((n_times, n_vis), dtype=np.complex128)
    for t in range(n_times):
        a[t, t * per:(t + 1) * per] = 1.0
    s = math.radians(fwhm_deg) / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    off = np.radians(np.linspace(-0.5 * drift_deg, 0.5 * drift_deg, n_times))
    centres = np.stack([np.sin(off), np.zeros(n_times), np.cos(off)], axis=1)
    d2 = ((xyz[None, :, :] - centres[:, None, :]) ** 2).sum(-1)
    b = np.exp(-d2 / (2.0 * s * s)).astype(np.complex128)
    return a, b


def noise_for_snr(signal_power_sum: float, m: int, snr_db: float,
                  rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian noise n ~ CN(0, s2) of length m with
    s2 = signal_power_sum / (m * 10^(snr_db/10))."""
    s2 = signal_power_sum / (m * 10.0 ** (snr_db / 10.0))
    return math.sqrt(s2 / 2.0) * (rng.standard_normal(m) + 1j * rng.standard_normal(m))


def sample_rows(n: int, k: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of ``min(k, n)`` distinct output indices."""
    rng = np.random.default_rng(seed)
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
