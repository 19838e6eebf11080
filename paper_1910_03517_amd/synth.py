"""Seeded synthetic camera rigs.

Input generation only: a periodic panorama (sky / ground gradients, three
low-frequency sinusoids, Gaussian sensor noise) cut into the cameras of a
ring, then distorted per camera by an exposure gain and per-channel white
balance gains (optionally a gamma curve).  It holds none of the correction
method's arithmetic, so both the oracle-based tests and the HIP path may use
it.  The paper's own footage is not available; these scenes stand in for a
ring of 1920x1080 remote-tower cameras looking at sky above ground.

Randomness: numpy.random.default_rng([1910, config_id, frame, ring, ...]).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SKY_TOP = (70.0, 110.0, 170.0)
SKY_HORIZON = (150.0, 170.0, 190.0)
GROUND_HORIZON = (90.0, 100.0, 70.0)
GROUND_BOTTOM = (50.0, 60.0, 40.0)
HORIZON = 0.55
SIN_AMP = 8.0


@dataclass(frozen=True)
class CamSpec:
    width: int
    height: int
    channels: int = 3
    bit_depth: int = 8
    ring: int = 0
    pos: int = 0

    @property
    def dtype(self):
        return np.uint8 if self.bit_depth == 8 else np.uint16


@dataclass
class RigSpec:
    name: str
    config_id: int
    cams: list = field(default_factory=list)

    @property
    def n_pixels(self) -> int:
        return sum(c.width * c.height for c in self.cams)

    @property
    def rings(self) -> list[int]:
        return sorted({c.ring for c in self.cams})


def ring_of(n: int, width: int, height: int, channels: int = 3, bit_depth: int = 8,
            ring: int = 0) -> list[CamSpec]:
    return [CamSpec(width, height, channels, bit_depth, ring, p) for p in range(n)]


def single_vga() -> RigSpec:
    """One 640x480 RGB camera (a ring of one)."""
    return RigSpec("1x640x480 rgb8", 1, ring_of(1, 640, 480))


def rig14_1080p() -> RigSpec:
    """14 cameras of 1920x1080 RGB, about 29 MPix per frame-set."""
    return RigSpec("14x1920x1080 rgb8", 2, ring_of(14, 1920, 1080))


def uneven_rig() -> RigSpec:
    """4x4096x2160 RGB + 8x1920x1080 RGB + 4x640x512 uint16 IR, three rings."""
    cams = (ring_of(4, 4096, 2160, ring=0) + ring_of(8, 1920, 1080, ring=1)
            + ring_of(4, 640, 512, channels=1, bit_depth=16, ring=2))
    return RigSpec("4x4096x2160 rgb8 + 8x1920x1080 rgb8 + 4x640x512 u16", 4, cams)


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng([1910, *key])


def scene_rgb(height: int, width: int, rng: np.random.Generator, noise_sigma: float = 4.0,
              no_clip: bool = False, phases: np.ndarray | None = None) -> np.ndarray:
    """Periodic-in-x RGB panorama, uint8 (height, width, 3).  `phases` of the
    three sinusoids (drawn from rng when None); the noise comes from rng."""
    hz = int(round(HORIZON * height))
    rows = np.zeros((height, 3), np.float32)
    t_sky = np.arange(hz, dtype=np.float32) / max(hz - 1, 1)
    t_gnd = np.arange(height - hz, dtype=np.float32) / max(height - hz - 1, 1)
    for c in range(3):
        rows[:hz, c] = SKY_TOP[c] + (SKY_HORIZON[c] - SKY_TOP[c]) * t_sky
        rows[hz:, c] = GROUND_HORIZON[c] + (GROUND_BOTTOM[c] - GROUND_HORIZON[c]) * t_gnd
    if phases is None:
        phases = rng.uniform(0.0, 2.0 * np.pi, 3)
    x = np.arange(width, dtype=np.float64)
    wave = sum(SIN_AMP * np.sin(2.0 * np.pi * m * x / width + phases[m - 1]) for m in (1, 2, 3))
    img = rows[:, None, :] + wave.astype(np.float32)[None, :, None]
    if no_clip:
        img = 16.0 + (img - 16.0) * np.float32(80.0 / 198.0)
    img += rng.standard_normal(img.shape, dtype=np.float32) * np.float32(noise_sigma)
    lo, hi = (16.0, 96.0) if no_clip else (0.0, 255.0)
    return np.clip(np.rint(img), lo, hi).astype(np.uint8)


def scene_ir(height: int, width: int, rng: np.random.Generator, noise_sigma: float = 1024.0,
             phases: np.ndarray | None = None) -> np.ndarray:
    """Periodic-in-x single-channel 16-bit panorama rescaled to [8000, 40000]."""
    hz = int(round(HORIZON * height))
    rows = np.zeros(height, np.float32)
    rows[:hz] = np.linspace(0.2, 0.8, hz, dtype=np.float32) if hz else rows[:0]
    rows[hz:] = np.linspace(0.7, 0.3, height - hz, dtype=np.float32) if height > hz else rows[hz:]
    if phases is None:
        phases = rng.uniform(0.0, 2.0 * np.pi, 3)
    x = np.arange(width, dtype=np.float64)
    wave = sum(0.05 * np.sin(2.0 * np.pi * m * x / width + phases[m - 1]) for m in (1, 2, 3))
    base = rows[:, None] + wave.astype(np.float32)[None, :]
    img = 8000.0 + np.clip(base, 0.0, 1.0) * 32000.0
    img = img.astype(np.float32) + rng.standard_normal(img.shape, dtype=np.float32) * np.float32(noise_sigma)
    return np.clip(np.rint(img), 0, 65535).astype(np.uint16)[:, :, None]


def draw_gains(n: int, channels: int, rng: np.random.Generator) -> np.ndarray:
    """Per-camera, per-channel gain g_k * wb_kc with g ~ U[0.5, 2], wb ~ U[0.8, 1.25]."""
    g = rng.uniform(0.5, 2.0, n)
    wb = rng.uniform(0.8, 1.25, (n, channels))
    return g[:, None] * wb


def drifted(gains: np.ndarray, frame: int, rng_key: tuple, period: int = 300,
            amp: float = 0.15) -> np.ndarray:
    """gains * exp(amp sin(2 pi t / period + phi)), phases fixed per camera and channel."""
    phi = _rng(*rng_key).uniform(0.0, 2.0 * np.pi, gains.shape)
    return gains * np.exp(amp * np.sin(2.0 * np.pi * frame / period + phi))


def distort(frame: np.ndarray, gain: np.ndarray, bit_depth: int, gamma: np.ndarray | None = None) -> np.ndarray:
    """y = clamp(round(gain_c * x)) per channel; optional gamma 255 (x / 255)^gamma first."""
    maxv = float((1 << bit_depth) - 1)
    x = frame.astype(np.float32)
    if gamma is not None:
        x = maxv * np.power(x / np.float32(maxv), gamma.astype(np.float32)[None, None, :])
    y = np.rint(x * gain.astype(np.float32)[None, None, :])
    return np.clip(y, 0.0, maxv).astype(frame.dtype)


def cut(pano: np.ndarray, widths: list[int]) -> list[np.ndarray]:
    out, x0 = [], 0
    for w in widths:
        out.append(np.ascontiguousarray(pano[:, x0:x0 + w]))
        x0 += w
    return out


@dataclass(frozen=True)
class MovingObject:
    """A textured rectangle (a vehicle seen from the tower) moving along the
    panorama of one ring: its left edge is at x0 + speed * frame (periodic in
    x), rows [y0, y0 + h), colour rgb plus a seeded stripe pattern."""
    x0: float
    y0: int
    w: int
    h: int
    speed: float
    rgb: tuple = (235.0, 40.0, 30.0)
    ring: int = 0

    def draw(self, pano: np.ndarray, frame: int) -> None:
        H, W = pano.shape[:2]
        x = int(round(self.x0 + self.speed * frame)) % W
        cols = (np.arange(self.w) + x) % W
        rows = np.arange(self.y0, min(self.y0 + self.h, H))
        stripes = (np.arange(self.w) // 8) % 2 * 25.0
        for c in range(min(3, pano.shape[2])):
            patch = np.clip(self.rgb[c] - stripes[None, :] + np.zeros((rows.size, 1)), 0, 255)
            pano[np.ix_(rows, cols, [c])] = np.rint(patch)[:, :, None].astype(pano.dtype)


def seam_crossing(rig: RigSpec, cam_pos: int = 0, speed: float = 24.0, frames: int = 12,
                  rows=(0.62, 0.70), width_frac: float = 0.08) -> MovingObject:
    """An object that crosses the seam between ring-0 positions cam_pos and
    cam_pos + 1 in the ground region, half way through `frames` frames."""
    cams = sorted((c for c in rig.cams if c.ring == 0), key=lambda c: c.pos)
    seam = sum(c.width for c in cams[:cam_pos + 1])
    h = cams[0].height
    w = max(4, int(round(width_frac * cams[0].width)))
    y0 = int(rows[0] * h)
    return MovingObject(x0=seam - w / 2 - speed * frames / 2, y0=y0, w=w, h=max(2, int((rows[1] - rows[0]) * h)),
                        speed=speed)


def rig_frames(rig: RigSpec, frame: int = 0, drift: bool = False, seed: int = 0,
               gamma: bool = False, no_clip: bool = False, distortion: bool = True,
               objects: tuple = (), noise_sigma: float = 4.0) -> list[np.ndarray]:
    """Distorted frames of every camera of `rig` for frame index `frame`.

    Gains and the scene are drawn once per (rig, seed); with drift the gains
    vary smoothly over a 300-frame period.  Sensor noise is redrawn for every
    frame.  `objects`
    (MovingObject) are drawn into their ring's panorama before it is cut and
    distorted.
    """
    frames: list[np.ndarray | None] = [None] * len(rig.cams)
    for ring in rig.rings:
        idx = sorted((c.pos, i) for i, c in enumerate(rig.cams) if c.ring == ring)
        idx = [i for _, i in idx]
        cams = [rig.cams[i] for i in idx]
        h = cams[0].height
        widths = [c.width for c in cams]
        rng = _rng(rig.config_id, seed, frame, ring)
        # The scene is fixed per (rig, seed, ring); the sensor noise is drawn per frame.
        phases = _rng(rig.config_id, seed, 30_000 + ring).uniform(0.0, 2.0 * np.pi, 3)
        if cams[0].bit_depth == 8:
            pano = scene_rgb(h, sum(widths), rng, noise_sigma=noise_sigma, no_clip=no_clip, phases=phases)
        else:
            pano = scene_ir(h, sum(widths), rng, phases=phases)
        for ob in objects:
            if ob.ring == ring and cams[0].bit_depth == 8:
                ob.draw(pano, frame)
        parts = cut(pano, widths)
        if cams[0].channels == 1 and parts[0].shape[2] == 3:
            parts = [p[:, :, :1].copy() for p in parts]
        grng = _rng(rig.config_id, seed, 10_000 + ring)
        gains = draw_gains(len(cams), cams[0].channels, grng)
        gam = grng.uniform(0.8, 1.25, (len(cams), cams[0].channels)) if gamma else None
        if drift:
            gains = drifted(gains, frame, (rig.config_id, seed, 20_000 + ring))
        for n, i in enumerate(idx):
            f = parts[n]
            if distortion:
                f = distort(f, gains[n], cams[n].bit_depth, None if gam is None else gam[n])
            frames[i] = f
    return frames  # type: ignore[return-value]


def tiny_frame(height: int, width: int, channels: int, bit_depth: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random frame for brute-force and fuzz cases."""
    dt = np.uint8 if bit_depth == 8 else np.uint16
    return rng.integers(0, 1 << bit_depth, (height, width, channels), dtype=np.int64).astype(dt)


def mlp_init(seed: int, n_in: int = 576, n_hid: int = 256, n_out: int = 6) -> dict:
    """Seeded He initialisation of the surrogate MLP (weights N(0, 2/fan_in), zero biases), float32."""
    rng = _rng(77, seed)
    f = np.float32
    return {"w1": (rng.standard_normal((n_in, n_hid)) * np.sqrt(2.0 / n_in)).astype(f), "b1": np.zeros(n_hid, f),
            "w2": (rng.standard_normal((n_hid, n_hid)) * np.sqrt(2.0 / n_hid)).astype(f), "b2": np.zeros(n_hid, f),
            "w3": (rng.standard_normal((n_hid, n_out)) * np.sqrt(2.0 / n_hid)).astype(f), "b3": np.zeros(n_out, f)}


def distort_device(base, gains: np.ndarray, cams, out) -> None:
    """Device-side gain distortion of undistorted frames (training-data synthesis):
    out = clamp(round(gain_kc * x)) per camera and channel, on torch tensors of
    shape (H, pitch) bytes holding each camera's rows (8-bit cameras only)."""
    import torch
    for k, (b, o, c) in enumerate(zip(base, out, cams)):
        rb = c.width * c.channels
        x = b[:, :rb].reshape(c.height, c.width, c.channels).to(torch.float32)
        g = torch.as_tensor(np.asarray(gains[k], np.float32), device=x.device)
        y = torch.clamp(torch.round(x * g), 0, 255).to(torch.uint8)
        o[:, :rb].copy_(y.reshape(c.height, rb))
