"""Seeded synthetic scenes and probe grids: inputs only.

This module builds triangle meshes, per-triangle albedos, light paths, vertex
animation and probe-grid descriptors for the probe-update workloads. It holds
none of the probe-update arithmetic (no ray generation, shading, detection,
allocation or blending). The GPU library's tests and the CPU oracle both
consume its arrays, so every array it returns is float32/int32 exactly as the
library receives it.

The paper's own assets (Bistro, Sponza, Buddha) are not available; these
generators stand in for them with the paper's grid shapes, texel resolutions
and dynamic events (moving lights, moving geometry).

All randomness comes from numpy's PCG64 with seed ``SEED_BASE + k``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 0xAD610000


@dataclasses.dataclass
class Scene:
    name: str
    positions: np.ndarray          # [V,3] float32
    indices: np.ndarray            # [T,3] int32
    albedo: np.ndarray             # [T,3] float32
    light_a: np.ndarray            # [L,3] float32, light position at frame 0
    light_b: np.ndarray            # [L,3] float32, light position at the last frame
    light_intensity: np.ndarray    # [L,3] float32, RGB intensity
    sky: np.ndarray                # [3] float32
    grid_origin: np.ndarray        # [3] float32, centre of probe (0,0,0)
    grid_spacing: np.ndarray       # [3] float32
    grid_dims: np.ndarray          # [3] int32
    frames: int
    # Optional vertical bobbing of a vertex prefix [0, anim_vertices):
    # dy(frame) = amp * sin(2*pi*freq*frame/fps + phase), one triple per group
    # of ``anim_group`` consecutive vertices.
    anim_vertices: int = 0
    anim_group: int = 8
    anim_amp: Optional[np.ndarray] = None
    anim_freq: Optional[np.ndarray] = None
    anim_phase: Optional[np.ndarray] = None
    fps: float = 60.0

    @property
    def num_probes(self) -> int:
        return int(np.prod(self.grid_dims.astype(np.int64)))

    @property
    def num_triangles(self) -> int:
        return int(self.indices.shape[0])

    @property
    def num_lights(self) -> int:
        return int(self.light_intensity.shape[0])

    def light_positions(self, frame: int) -> np.ndarray:
        """Linear light path, evaluated in float64 and rounded to float32."""
        if self.frames <= 1:
            f = 0.0
        else:
            f = min(max(frame, 0), self.frames - 1) / (self.frames - 1)
        a = self.light_a.astype(np.float64)
        b = self.light_b.astype(np.float64)
        return (a + (b - a) * f).astype(np.float32)

    def write_animated(self, frame: int, out: np.ndarray) -> None:
        """Write the animated vertex prefix of ``frame`` into ``out`` (a full
        [V,3] float32 buffer); vertices past the prefix are left untouched."""
        if self.anim_vertices == 0:
            return
        t = frame / self.fps
        dy = (self.anim_amp.astype(np.float64)
              * np.sin(2.0 * math.pi * self.anim_freq.astype(np.float64) * t
                       + self.anim_phase.astype(np.float64)))
        dy = np.repeat(dy, self.anim_group)[: self.anim_vertices]
        out[: self.anim_vertices, 1] = (
            self.positions[: self.anim_vertices, 1].astype(np.float64) + dy).astype(np.float32)

    def positions_at(self, frame: int) -> np.ndarray:
        """Vertex positions at ``frame`` (animated prefix bobbing in y)."""
        if self.anim_vertices == 0:
            return self.positions
        pos = self.positions.copy()
        n_groups = self.anim_vertices // self.anim_group
        t = frame / self.fps
        dy = (self.anim_amp.astype(np.float64)
              * np.sin(2.0 * math.pi * self.anim_freq.astype(np.float64) * t
                       + self.anim_phase.astype(np.float64)))
        dy = np.repeat(dy, self.anim_group)[: self.anim_vertices]
        pos[: self.anim_vertices, 1] = (
            self.positions[: self.anim_vertices, 1].astype(np.float64) + dy
        ).astype(np.float32)
        assert n_groups * self.anim_group == self.anim_vertices
        return pos


# ---------------------------------------------------------------- geometry

_CORNERS = np.array([[(i >> 0) & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)],
                    dtype=np.float64)


def _box_faces(outward: bool) -> np.ndarray:
    """12 triangles (local vertex indices 0..7) of an axis-aligned box.

    Winding is chosen so that (v1-v0)x(v2-v0) points out of the box when
    ``outward`` is true and into it otherwise.
    """
    tris = []
    for axis in range(3):
        for side in (0, 1):
            quad = [i for i in range(8) if ((i >> axis) & 1) == side]
            # quad corners ordered around the face
            a, b = [x for x in range(3) if x != axis]
            ring = sorted(quad, key=lambda i: math.atan2(_CORNERS[i][b] - 0.5,
                                                         _CORNERS[i][a] - 0.5))
            for t in ((ring[0], ring[1], ring[2]), (ring[0], ring[2], ring[3])):
                v0, v1, v2 = (_CORNERS[k] for k in t)
                n = np.cross(v1 - v0, v2 - v0)
                want = (1.0 if side == 1 else -1.0) * (1.0 if outward else -1.0)
                if n[axis] * want < 0:
                    t = (t[0], t[2], t[1])
                tris.append(t)
    return np.array(tris, dtype=np.int32)


_BOX_OUT = _box_faces(True)
_BOX_IN = _box_faces(False)


def _boxes(lo: np.ndarray, hi: np.ndarray, outward: bool = True):
    """Vertices [8N,3] and triangles [12N,3] for N boxes (float64 in)."""
    n = lo.shape[0]
    verts = lo[:, None, :] + _CORNERS[None, :, :] * (hi - lo)[:, None, :]
    faces = (_BOX_OUT if outward else _BOX_IN)[None, :, :] + 8 * np.arange(n)[:, None, None]
    return verts.reshape(-1, 3), faces.reshape(-1, 3).astype(np.int32)


def _grid_over(lo, hi, dims):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    dims = np.asarray(dims, np.int64)
    spacing = (hi - lo) / dims
    origin = lo + 0.5 * spacing
    return origin.astype(np.float32), spacing.astype(np.float32), dims.astype(np.int32)


# ---------------------------------------------------------------- scenes

def cornell() -> Scene:
    """Closed Cornell-like room [0,1]^3 with two boxes: 36 triangles.

    Probes 4x4x4 at 0.125 + 0.25*k; three of them lie inside the boxes.
    """
    room_v, room_t = _boxes(np.zeros((1, 3)), np.ones((1, 3)), outward=False)
    lo = np.array([[0.15, 0.0, 0.5], [0.55, 0.0, 0.15]])
    hi = np.array([[0.45, 0.6, 0.8], [0.85, 0.3, 0.45]])
    box_v, box_t = _boxes(lo, hi, outward=True)
    pos = np.concatenate([room_v, box_v]).astype(np.float32)
    idx = np.concatenate([room_t, box_t + room_v.shape[0]]).astype(np.int32)
    alb = np.full((idx.shape[0], 3), 0.75, np.float32)
    # room walls: x=0 (left) red, x=1 (right) green
    for t in range(12):
        xs = pos[room_t[t], 0]
        if np.all(xs == 0.0):
            alb[t] = (0.75, 0.1, 0.1)
        elif np.all(xs == 1.0):
            alb[t] = (0.1, 0.75, 0.1)
    lp = np.array([[0.5, 0.95, 0.5]], np.float32)
    return Scene(
        name="cornell", positions=pos, indices=idx, albedo=alb,
        light_a=lp, light_b=lp.copy(), light_intensity=np.ones((1, 3), np.float32),
        sky=np.zeros(3, np.float32),
        grid_origin=np.full(3, 0.125, np.float32), grid_spacing=np.full(3, 0.25, np.float32),
        grid_dims=np.array([4, 4, 4], np.int32), frames=8)


def tunnel(seed: int = SEED_BASE + 1, rings: int = 256, sides: int = 160,
           n_boxes: int = 1500, frames: int = 60) -> Scene:
    """Tube along +z of random-radius rings plus random boxes (~100k triangles).

    Two point lights (I = 5) move on seeded straight paths inside the tube.
    Probe grid 16x8x16 over the tube's bounding box.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = rng.uniform(1.5, 2.5, size=rings)
    ang = 2.0 * math.pi * np.arange(sides) / sides
    z = 0.25 * np.arange(rings)
    ring_v = np.stack([radius[:, None] * np.cos(ang)[None, :],
                       radius[:, None] * np.sin(ang)[None, :],
                       np.broadcast_to(z[:, None], (rings, sides))], axis=-1).reshape(-1, 3)
    a = np.arange(rings - 1)[:, None]
    k = np.arange(sides)[None, :]
    k1 = (k + 1) % sides
    v00 = a * sides + k
    v01 = a * sides + k1
    v10 = (a + 1) * sides + k
    v11 = (a + 1) * sides + k1
    tri = np.concatenate([np.stack([v00, v01, v11], -1).reshape(-1, 3),
                          np.stack([v00, v11, v10], -1).reshape(-1, 3)])
    # orient so that the geometric normal points towards the tube axis
    p0 = ring_v[tri[:, 0]]
    n = np.cross(ring_v[tri[:, 1]] - p0, ring_v[tri[:, 2]] - p0)
    inward = -(p0 * np.array([1.0, 1.0, 0.0]))
    flip = np.einsum("ij,ij->i", n, inward) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    tube_t = tri.astype(np.int32)
    rmax = float(radius.max())
    bb_lo = np.array([-rmax, -rmax, 0.0])
    bb_hi = np.array([rmax, rmax, float(z[-1])])
    edge = rng.uniform(0.1, 0.5, size=(n_boxes, 3))
    centre = rng.uniform(bb_lo, bb_hi, size=(n_boxes, 3))
    box_v, box_t = _boxes(centre - 0.5 * edge, centre + 0.5 * edge)
    box_alb = rng.uniform(0.2, 0.9, size=(n_boxes, 3))
    pos = np.concatenate([ring_v, box_v]).astype(np.float32)
    idx = np.concatenate([tube_t, box_t + ring_v.shape[0]]).astype(np.int32)
    alb = np.concatenate([np.full((tube_t.shape[0], 3), 0.6),
                          np.repeat(box_alb, 12, axis=0)]).astype(np.float32)
    # lights: straight paths inside radius 1.2, z in [2, zmax-2]
    def disc_points(m):
        r = 1.2 * np.sqrt(rng.uniform(0.0, 1.0, m))
        th = rng.uniform(0.0, 2.0 * math.pi, m)
        zz = rng.uniform(2.0, float(z[-1]) - 2.0, m)
        return np.stack([r * np.cos(th), r * np.sin(th), zz], -1)
    la = disc_points(2).astype(np.float32)
    lb = disc_points(2).astype(np.float32)
    origin, spacing, dims = _grid_over(bb_lo, bb_hi, (16, 8, 16))
    return Scene(
        name="tunnel", positions=pos, indices=idx, albedo=alb,
        light_a=la, light_b=lb, light_intensity=np.full((2, 3), 5.0, np.float32),
        sky=np.zeros(3, np.float32), grid_origin=origin, grid_spacing=spacing,
        grid_dims=dims, frames=frames)


def box_field(seed: int = SEED_BASE + 2, lattice: int = 288, pitch: float = 0.25,
              dims=(64, 16, 64), n_lights: int = 3, frames: int = 60,
              anim_fraction: float = 0.05, grid_height: float = 4.8) -> Scene:
    """Lattice of boxes on a ground quad: lattice^2 * 12 + 2 triangles.

    The default (288^2 boxes) gives 995,330 triangles. A seeded 5% of the
    boxes bob vertically; their vertices form the prefix of the vertex array
    so that a refit uploads one contiguous range.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = lattice * lattice
    ia, ib = np.meshgrid(np.arange(lattice), np.arange(lattice), indexing="ij")
    cx = (ia.reshape(-1) + 0.5) * pitch
    cz = (ib.reshape(-1) + 0.5) * pitch
    wx = rng.uniform(0.05, 0.2, nb)
    wz = rng.uniform(0.05, 0.2, nb)
    h = rng.uniform(0.1, 4.0, nb)
    alb_box = rng.uniform(0.2, 0.9, size=(nb, 3))
    n_anim = int(round(anim_fraction * nb))
    anim_ids = rng.choice(nb, size=n_anim, replace=False)
    order = np.concatenate([np.sort(anim_ids), np.setdiff1d(np.arange(nb), anim_ids)])
    cx, cz, wx, wz, h, alb_box = (x[order] for x in (cx, cz, wx, wz, h, alb_box))
    lo = np.stack([cx - 0.5 * wx, np.zeros(nb), cz - 0.5 * wz], -1)
    hi = np.stack([cx + 0.5 * wx, h, cz + 0.5 * wz], -1)
    box_v, box_t = _boxes(lo, hi)
    ext = lattice * pitch
    g = np.array([[-1.0, 0.0, -1.0], [ext + 1.0, 0.0, -1.0],
                  [-1.0, 0.0, ext + 1.0], [ext + 1.0, 0.0, ext + 1.0]])
    gt = np.array([[0, 2, 1], [1, 2, 3]])  # normal +y
    pos = np.concatenate([box_v, g]).astype(np.float32)
    idx = np.concatenate([box_t, gt + box_v.shape[0]]).astype(np.int32)
    alb = np.concatenate([np.repeat(alb_box, 12, axis=0), np.full((2, 3), 0.5)]).astype(np.float32)
    amp = rng.uniform(0.1, 0.5, n_anim).astype(np.float32)
    freq = rng.uniform(0.25, 1.0, n_anim).astype(np.float32)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_anim).astype(np.float32)
    def light_points(m):
        xz = rng.uniform(0.1 * ext, 0.9 * ext, size=(m, 2))
        y = rng.uniform(5.0, 8.0, m)
        return np.stack([xz[:, 0], y, xz[:, 1]], -1).astype(np.float32)
    la = light_points(n_lights)
    lb = light_points(n_lights)
    inten = (np.array([[30.0, 27.0, 24.0], [24.0, 27.0, 30.0], [27.0, 30.0, 24.0]])[:n_lights]
             * (ext / 72.0) ** 2).astype(np.float32)
    origin, spacing, dims_ = _grid_over((0.0, 0.0, 0.0), (ext, grid_height, ext), dims)
    return Scene(
        name="box_field", positions=pos, indices=idx, albedo=alb,
        light_a=la, light_b=lb, light_intensity=inten, sky=np.zeros(3, np.float32),
        grid_origin=origin, grid_spacing=spacing, grid_dims=dims_, frames=frames,
        anim_vertices=8 * n_anim, anim_group=8, anim_amp=amp, anim_freq=freq,
        anim_phase=phase)


def sample_probes(num_probes: int, k: int = 512, seed: int = SEED_BASE + 3) -> np.ndarray:
    """Probe indices sampled uniformly without replacement, ascending."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(num_probes, size=min(k, num_probes), replace=False)).astype(np.int32)


@dataclasses.dataclass
class Stream:
    """One serving stream: a scene, a budget and a Poisson arrival process."""
    scene: Scene
    budget: int
    rate_hz: float
    arrivals: np.ndarray  # arrival times in seconds, ascending


def serving_streams(seed: int = SEED_BASE + 4, n_streams: int = 32,
                    duration_s: float = 10.0, tri_range=(10_000, 500_000),
                    probe_range=(512, 32768)) -> list:
    """Serving mix: stream sizes log-uniform in triangles and probes.

    Each stream is a box field whose lattice gives the drawn triangle count,
    a probe grid of dims (x, x/4, x) near the drawn probe count, 1-3 moving
    lights, budget 128 rays per probe, and Poisson arrivals at U[30,120] Hz.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(n_streams):
        tris = math.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1])))
        probes = math.exp(rng.uniform(math.log(probe_range[0]), math.log(probe_range[1])))
        lattice = max(4, int(round(math.sqrt((tris - 2) / 12.0))))
        x = max(4, int(round((4.0 * probes) ** (1.0 / 3.0) / 4.0)) * 4)
        n_lights = int(rng.integers(1, 4))
        rate = float(rng.uniform(30.0, 120.0))
        gaps = rng.exponential(1.0 / rate, size=int(rate * duration_s * 2) + 16)
        t = np.cumsum(gaps)
        t = t[t < duration_s]
        sc = box_field(seed=SEED_BASE + 100 + s, lattice=lattice, dims=(x, x // 4, x),
                       n_lights=n_lights, frames=max(2, len(t)))
        out.append(Stream(scene=sc, budget=128 * sc.num_probes, rate_hz=rate, arrivals=t))
    return out


CONFIGS = {
    "cornell": cornell,
    "tunnel": tunnel,
    "box_field": box_field,
}
