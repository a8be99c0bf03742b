"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against a closed form, a published test vector,
a number printed in the paper, brute force on tiny inputs, or an invariant of
the mathematics, chosen so that a plausible slip (a dropped term, a wrong
sign or index, a transposed operand) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G64 = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------- O2: RNG

def test_splitmix64_published_vectors():
    for seed, k, out in _read_golden("splitmix64.txt"):
        state = (int(seed) + int(k) * G64) & M64
        assert oracle.splitmix64(state) == int(out)


def test_uniforms_are_24_bit_and_in_range():
    L = oracle.lib()
    for k in range(200):
        key = L.orc_key(1, 2, k, 3, 4)
        u = L.orc_uniform(key, 1)
        assert 0.0 <= u < 1.0
        assert (u * 2 ** 24) == int(u * 2 ** 24)


# ----------------------------------------------------- O2: rotations, SF

def test_frame_rotation_is_orthonormal_fp32():
    for t in range(50):
        R = oracle.frame_rotation(12345, t).astype(np.float64)
        assert np.abs(R.T @ R - np.eye(3)).max() < 1e-6
        assert abs(np.linalg.det(R) - 1.0) < 1e-6
    # distinct frames give distinct rotations
    assert not np.array_equal(oracle.frame_rotation(1, 0), oracle.frame_rotation(1, 1))


def test_frame_rotation_uniform_on_so3():
    # For a Haar-random rotation E[R] = 0 and E[trace R] = 0.
    Rs = np.stack([oracle.frame_rotation(99, t).astype(np.float64) for t in range(4000)])
    assert np.abs(Rs.mean(axis=0)).max() < 0.05
    assert abs(np.trace(Rs, axis1=1, axis2=2).mean()) < 0.1


@pytest.mark.parametrize("n", [8, 64, 257, 1024])
def test_spherical_fibonacci_properties(n):
    I = np.eye(3, dtype=np.float32)
    d = oracle.sf_dirs(n, I)
    # z_j = 1 - (2j+1)/n exactly (identity rotation)
    j = np.arange(n)
    assert np.array_equal(d[:, 2], 1.0 - (2.0 * j + 1.0) / n)
    assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() < 1e-15
    # near-uniform: the mean direction is O(1/n)
    assert np.linalg.norm(d.mean(axis=0)) < 2.0 / n
    # equal-area in z (Archimedes): each z-band of the sphere holds its share
    counts, _ = np.histogram(d[:, 2], bins=4, range=(-1, 1))
    assert np.all(np.abs(counts - n / 4) <= 1)
    # golden-angle azimuth: successive points differ by 2*pi*(1 - 1/phi)
    phi = np.arctan2(d[:, 1], d[:, 0])
    dphi = np.mod(phi[1:] - phi[:-1], 2 * np.pi)
    golden = 2 * np.pi * (2 - (1 + 5 ** 0.5) / 2)
    assert np.allclose(np.minimum(dphi, 2 * np.pi - dphi), golden, atol=1e-9)


@pytest.mark.parametrize("n", [1, 7, 64, 65, 100, 127, 128, 129, 300, 2047, 2048, 4097])
def test_ray_point_strata(n):
    # brute force of the stratified assignment: the residue classes of the
    # point indices modulo C = ceil(n/64), each ascending, concatenated
    C = -(-n // 64)
    order = [p for c in range(C) for p in range(c, n, C)]
    got = [oracle.ray_point(j, n) for j in range(n)]
    assert got == order
    assert sorted(got) == list(range(n))  # a permutation: the probe still traces the whole set
    if n <= 64:
        assert got == list(range(n))
    # each stratum (at most 64 rays) spans the sphere: its mean z is small,
    # unlike that of as many consecutive points (a thin band in z)
    d = oracle.probe_ray_dirs(n, np.eye(3, dtype=np.float32))
    if n >= 128:
        m = -(-n // C)  # stratum 0's size
        assert m <= 64
        assert np.abs(d[:m, 2].mean()) < 0.1
        assert oracle.sf_dirs(n, np.eye(3, dtype=np.float32))[:m, 2].mean() > 0.4


def test_probe_ray_directions_are_the_point_set():
    R = oracle.frame_rotation(3, 1)
    for n in (8, 200, 1000):
        a = oracle.probe_ray_dirs(n, R)
        b = oracle.sf_dirs(n, R)
        assert np.array_equal(a[np.argsort([oracle.ray_point(j, n) for j in range(n)])], b)


def test_sf_rotation_applies_matrix():
    R = oracle.frame_rotation(5, 3)
    d0 = oracle.sf_dirs(33, np.eye(3, dtype=np.float32))
    d1 = oracle.sf_dirs(33, R)
    assert np.abs(d1 - d0 @ R.astype(np.float64).T).max() < 1e-14


def test_pilot_directions_in_octant_and_pair_stable():
    for probe in range(20):
        for k in range(8):
            for pair in range(3):
                d = oracle.pilot_dir(7, probe, k, pair)
                assert abs(np.linalg.norm(d) - 1.0) < 1e-12
                sx = -1 if k & 1 else 1
                sy = -1 if k & 2 else 1
                sz = -1 if k & 4 else 1
                assert d[0] * sx >= 0 and d[1] * sy >= 0 and d[2] * sz >= 0
            # same pair -> same direction; the frame index only enters via pair
    assert np.array_equal(oracle.pilot_dir(7, 3, 2, 5), oracle.pilot_dir(7, 3, 2, 5))
    assert not np.array_equal(oracle.pilot_dir(7, 3, 2, 5), oracle.pilot_dir(7, 3, 2, 6))


def test_pilot_directions_uniform_within_octant():
    # Folded uniform sphere points: each |component| has mean 1/2.
    ds = np.array([np.abs(oracle.pilot_dir(11, p, 0, 0)) for p in range(6000)])
    assert np.abs(ds.mean(axis=0) - 0.5).max() < 0.02


# -------------------------------------------------------- O1: octahedral

def test_octahedral_axes_closed_form():
    cases = {(1, 0, 0): (1, 0), (-1, 0, 0): (-1, 0), (0, 1, 0): (0, 1), (0, -1, 0): (0, -1),
             (0, 0, 1): (0, 0)}
    for d, uv in cases.items():
        assert np.allclose(oracle.oct_encode(np.array(d, float)), uv, atol=1e-15)
    # the south pole sits at the four corners
    assert np.allclose(np.abs(oracle.oct_encode(np.array([0.0, 0.0, -1.0]))), [1, 1])
    for c in [(1, 1), (-1, 1), (1, -1), (-1, -1)]:
        assert np.allclose(oracle.oct_decode(np.array(c, float)), [0, 0, -1], atol=1e-15)


def test_octahedral_round_trip():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for v in d:
        uv = oracle.oct_encode(v)
        assert abs(uv[0]) <= 1 and abs(uv[1]) <= 1
        if v[2] >= 0:
            assert abs(uv[0]) + abs(uv[1]) <= 1 + 1e-15
        assert np.abs(oracle.oct_decode(uv) - v).max() < 1e-15


@pytest.mark.parametrize("r", [6, 14])
def test_octahedral_bins_centres_and_coverage(r):
    # decode(centre of texel k) falls in texel k; encode(decode(centre)) = centre
    for iy in range(r):
        for ix in range(r):
            c = np.array([(ix + 0.5) / r * 2 - 1, (iy + 0.5) / r * 2 - 1])
            d = oracle.oct_decode(c)
            assert np.abs(oracle.oct_encode(d) - c).max() < 1e-14
            k, tie = oracle.oct_bin(d, r, 1e-6)
            assert k == iy * r + ix and not tie
    # every texel receives directions; solid angles of cells add up to 4*pi
    rng = np.random.default_rng(1)
    d = rng.normal(size=(60000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ks = np.array([oracle.oct_bin(v, r)[0] for v in d])
    cnt = np.bincount(ks, minlength=r * r)
    assert cnt.shape[0] == r * r and cnt.min() > 0
    # the map is not equal-area: cell solid angles vary (about 1.85x at 6x6)
    ratio = cnt.max() / cnt.min()
    assert 1.3 < ratio < 6.0


def test_octahedral_edge_identification():
    # (u,+-1) ~ (-u,+-1) and (+-1,v) ~ (+-1,-v) decode to the same direction
    for u in np.linspace(-1, 1, 41):
        for s in (-1.0, 1.0):
            assert np.abs(oracle.oct_decode([u, s]) - oracle.oct_decode([-u, s])).max() < 1e-15
            assert np.abs(oracle.oct_decode([s, u]) - oracle.oct_decode([s, -u])).max() < 1e-15


@pytest.mark.parametrize("r", [6, 14])
def test_border_fold_is_edge_mirror(r):
    """The source of a border texel is the mirror image, across the map edge,
    of the interior texel next to the border: the direction of the source's
    centre equals the adjacent texel's with x negated (top/bottom edge, which
    maps to the plane x = 0), y negated (left/right, plane y = 0) or both
    (corners, the south pole)."""
    def centre_dir(X, Y):
        return oracle.oct_decode([(X - 0.5) / r * 2 - 1, (Y - 0.5) / r * 2 - 1])
    w = r + 2
    for Y in range(w):
        for X in range(w):
            bx, by = X in (0, r + 1), Y in (0, r + 1)
            if not (bx or by):
                continue
            sx, sy = oracle.border_source(X, Y, r)
            assert 1 <= sx <= r and 1 <= sy <= r
            ax, ay = min(max(X, 1), r), min(max(Y, 1), r)  # adjacent interior texel
            m = np.array([-1.0 if by else 1.0, -1.0 if bx else 1.0, 1.0])
            assert np.abs(centre_dir(sx, sy) - m * centre_dir(ax, ay)).max() < 1e-14, (X, Y)
    # fold of a tile copies interior texels unchanged
    interior = np.arange(r * r * 2, dtype=np.float64)
    tile = oracle.fold_tile(interior, r, 2)
    assert np.array_equal(tile[1:r + 1, 1:r + 1].reshape(-1), interior)


# ------------------------------------------------------ O3: intersection

def _quad(x0, x1, y0, y1, z):
    pos = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return pos, idx


def test_axis_aligned_exact_t():
    pos, idx = _quad(-1, 1, -1, 1, 2.5)
    sc = oracle.OracleScene(pos, idx, np.ones((2, 3), np.float32), use_bvh=False)
    h = sc.closest_hit([0.25, 0.5, 0.0], [0.0, 0.0, 1.0], brute=True)
    assert h.t == 2.5 and h.tri in (0, 1)
    assert h.front == 0  # winding gives normal +z; ray along +z sees the back
    h = sc.closest_hit([0.25, 0.5, 5.0], [0.0, 0.0, -1.0], brute=True)
    assert h.t == 2.5 and h.front == 1
    h = sc.closest_hit([3.0, 0.0, 0.0], [0.0, 0.0, 1.0], brute=True)
    assert h.tri == -1 and math.isinf(h.t)


def test_bvh_equals_brute_force_on_tiny_scenes():
    rng = np.random.default_rng(3)
    tol = oracle.default_tol()
    for trial in range(8):
        nt = int(rng.integers(1, 65))
        pos = rng.uniform(-2, 2, size=(3 * nt, 3)).astype(np.float32)
        idx = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
        alb = np.ones((nt, 3), np.float32)
        bvh = oracle.OracleScene(pos, idx, alb, use_bvh=True)
        for _ in range(300):
            o = rng.uniform(-3, 3, 3)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            a = bvh.closest_hit(o, d, tol)
            b = bvh.closest_hit(o, d, tol, brute=True)
            assert (a.tri, a.t, a.front, a.tie) == (b.tri, b.t, b.front, b.tie)


def test_closest_hit_ties_break_to_lowest_index():
    pos1, idx1 = _quad(-1, 1, -1, 1, 1.0)
    pos = np.concatenate([pos1, pos1])
    idx = np.concatenate([idx1, idx1 + 4])[[2, 0, 3, 1]]  # duplicates, shuffled
    sc = oracle.OracleScene(pos, idx, np.ones((4, 3), np.float32), use_bvh=False)
    h = sc.closest_hit([0.3, -0.2, 0.0], [0.0, 0.0, 1.0], oracle.default_tol())
    assert h.t == 1.0 and h.tri == min(t for t in range(4) if True and t in (0, 1, 2, 3)
                                        and _contains(pos, idx[t], 0.3, -0.2))
    assert h.tie  # a second surface at the same depth is a tie


def _contains(pos, tri, x, y):
    a, b, c = pos[tri][:, :2].astype(np.float64)
    def s(p, q, r):
        return (p[0] - r[0]) * (q[1] - r[1]) - (q[0] - r[0]) * (p[1] - r[1])
    p = np.array([x, y])
    d1, d2, d3 = s(p, a, b), s(p, b, c), s(p, c, a)
    return not ((d1 < 0 or d2 < 0 or d3 < 0) and (d1 > 0 or d2 > 0 or d3 > 0))


def test_edge_and_near_miss_rays_are_ties():
    pos, idx = _quad(-1, 1, -1, 1, 1.0)
    sc = oracle.OracleScene(pos, idx, np.ones((2, 3), np.float32), use_bvh=False)
    tol = oracle.default_tol()
    # interior: no tie; on the shared diagonal: tie; just outside: tie
    assert not sc.closest_hit([0.5, -0.3, 0.0], [0, 0, 1.0], tol).tie
    assert sc.closest_hit([0.3, 0.3, 0.0], [0, 0, 1.0], tol).tie
    h = sc.closest_hit([1.0 + 1e-9, 0.0, 0.0], [0, 0, 1.0], tol)
    assert h.tri == -1 and h.tie
    h = sc.closest_hit([1.1, 0.0, 0.0], [0, 0, 1.0], tol)
    assert h.tri == -1 and not h.tie


# ----------------------------------------------------------- O4: shading

def test_pin1_uniform_sky_empty_scene():
    """Uniform sky, no triangles: every sampled texel holds the sky radiance
    exactly, depth texels hold tau_max and tau_max^2, counts = samples."""
    sc = scenes.cornell()
    empty = scenes.Scene(
        name="empty", positions=np.zeros((0, 3), np.float32), indices=np.zeros((0, 3), np.int32),
        albedo=np.zeros((0, 3), np.float32), light_a=np.zeros((0, 3), np.float32),
        light_b=np.zeros((0, 3), np.float32), light_intensity=np.zeros((0, 3), np.float32),
        sky=np.array([0.7, 1.3, 2.0], np.float32), grid_origin=sc.grid_origin,
        grid_spacing=sc.grid_spacing, grid_dims=np.array([2, 2, 2], np.int32), frames=4)
    vol = oracle.OracleVolume(empty, seed=5)
    total = np.zeros((8, 36))
    for f in range(3):
        out = vol.update(f, adaptive=False, n_uniform=97, keep_rays=True)
        for q in range(8):
            b = out["ray_base"][q]
            total[q] += np.bincount(out["irr_bin"][b:b + 97], minlength=36)
    sky = np.float32([0.7, 1.3, 2.0]).astype(np.float64)
    ri = vol.irr.reshape(8, 36, 3)
    hit = vol.irr_n > 0
    assert np.array_equal(vol.irr_n, np.minimum(total, 255).astype(np.uint8))
    assert np.all(ri[hit] == sky)
    dep = vol.dep.reshape(8, 196, 2)
    dh = vol.dep_n > 0
    assert np.all(dep[dh][:, 0] == vol.tau_max)
    assert np.all(dep[dh][:, 1] == vol.tau_max ** 2)
    # untouched texels keep their initial value 0
    assert np.all(ri[~hit] == 0) and np.all(dep[~dh] == 0)


def _plane_light_scene(H, rho, I, half=None):
    half = half if half is not None else 200.0 * H
    pos, idx = _quad(-half, half, -half, half, 0.0)  # normal +z (faces the light)
    sc = oracle.OracleScene(pos, idx, np.full((2, 3), rho, np.float32), use_bvh=False)
    sc.set_lights(np.array([[0.0, 0.0, H]], np.float32), np.full((1, 3), I, np.float32),
                  np.zeros(3, np.float32))
    return sc


def _downward_irradiance(sc, probe, s=1.0, n_theta=96, n_phi=6):
    # E = int L(w) cos(theta) dw over the lower hemisphere, Gauss-Legendre in
    # cos(theta), midpoint in phi (the setup is rotationally symmetric).
    x, w = np.polynomial.legendre.leggauss(n_theta)
    mu = 0.5 * (x + 1.0)
    wm = 0.5 * w
    E = 0.0
    for m, wt in zip(mu, wm):
        st = math.sqrt(max(0.0, 1 - m * m))
        acc = 0.0
        for k in range(n_phi):
            ph = 2 * math.pi * (k + 0.5) / n_phi
            d = np.array([st * math.cos(ph), st * math.sin(ph), -m])
            acc += sc.shade(probe, d, s).rgb[0]
        E += wt * m * (acc / n_phi) * 2 * math.pi
    return E


@pytest.mark.parametrize("H", [1.0, 2.0])
def test_pin2_point_light_over_plane_colocated(H):
    """Probe at the light, plane below: E = 2 rho I / (5 H^2)."""
    rho, I = 0.75, 3.0
    sc = _plane_light_scene(H, rho, I)
    E = _downward_irradiance(sc, np.array([0.0, 0.0, H]))
    exact = 2 * float(np.float32(rho)) * I / (5 * H * H)
    assert abs(E - exact) / exact < 1e-6


@pytest.mark.parametrize("h", [0.5, 3.0])
def test_pin2_point_light_over_plane_general_height(h):
    """Probe at height h, light at H: E = rho I H h^2 int du/((u+H^2)^1.5 (u+h^2)^2)."""
    rho, I, H = 0.5, 2.0, 1.5
    sc = _plane_light_scene(H, rho, I, half=400.0)
    E = _downward_irradiance(sc, np.array([0.0, 0.0, h]), n_theta=160)
    f = lambda u: 1.0 / ((u + H * H) ** 1.5 * (u + h * h) ** 2)
    integral, _ = integrate.quad(f, 0.0, np.inf, epsabs=0, epsrel=1e-12)
    exact = float(np.float32(rho)) * I * H * h * h * integral
    assert abs(E - exact) / exact < 1e-5


def test_pin9_direct_light_one_triangle_and_blocker():
    pos = np.array([[-5, 0, -5], [5, 0, -5], [0, 0, 5]], np.float32)  # y = 0 plane
    idx = np.array([[0, 2, 1]], np.int32)
    v = pos.astype(np.float64)
    n = np.cross(v[2] - v[0], v[1] - v[0])
    assert n[1] > 0  # normal +y
    sc = oracle.OracleScene(pos, idx, np.array([[0.6, 0.3, 0.9]], np.float32), use_bvh=False)
    lp = np.array([1.0, 2.0, 0.5])
    I = np.array([2.0, 4.0, 8.0])
    sc.set_lights(lp[None].astype(np.float32), I[None].astype(np.float32), np.zeros(3, np.float32))
    o = np.array([0.0, 1.0, 0.0])
    d = np.array([0.3, -1.0, 0.2])
    d /= np.linalg.norm(d)
    r = sc.shade(o, d, 1.0)
    x = o + (1.0 / -d[1]) * d
    L = lp - x
    cos = L[1] / np.linalg.norm(L)
    rho = np.array([0.6, 0.3, 0.9], np.float32).astype(np.float64)
    expect = rho / math.pi * I * cos / (L @ L)
    assert np.allclose(np.array(r.rgb), expect, rtol=1e-13, atol=0)
    assert r.shadow == 1 and r.front == 1
    # add a blocker between the hit point and the light
    bpos = np.concatenate([pos, np.array([[-9, 1.5, -9], [9, 1.5, -9], [0, 1.5, 9]], np.float32)])
    bidx = np.array([[0, 2, 1], [3, 4, 5]], np.int32)
    sc2 = oracle.OracleScene(bpos, bidx, np.ones((2, 3), np.float32), use_bvh=False)
    sc2.set_lights(lp[None].astype(np.float32), I[None].astype(np.float32), np.zeros(3, np.float32))
    r2 = sc2.shade(o, d, 1.0)
    assert r2.tri == 0 and r2.shadow == 0 and list(r2.rgb) == [0.0, 0.0, 0.0]
    # back face: zero radiance, distance kept
    r3 = sc.shade(np.array([0.0, -1.0, 0.0]), np.array([0.0, 1.0, 0.0]), 1.0)
    assert r3.front == 0 and r3.t == 1.0 and list(r3.rgb) == [0.0, 0.0, 0.0]
    # light below the surface: no contribution
    sc.set_lights(np.array([[0.0, -2.0, 0.0]], np.float32), I[None].astype(np.float32),
                  np.zeros(3, np.float32))
    assert list(sc.shade(o, d, 1.0).rgb) == [0.0, 0.0, 0.0]


# ------------------------------------------------------------- O7: blend

def test_pin6_hysteresis_matches_printed_table():
    """Alg. MovingAvgUpdate with N_max saturates at N_max/(N_max+1); the
    paper's table prints these as 0.98 (63) and 0.91 (10). With the real-valued
    N_max = h/(1-h), the saturated step 1-h reproduces that weight."""
    for name, nmax, printed in _read_golden("cache_hysteresis.txt"):
        nmax = int(nmax)
        h = nmax / (nmax + 1.0)
        assert round(h, 2) == float(printed)
        # past saturation the new sample's weight is 1/(N_max+1) = 1-h
        assert abs(oracle.blend_alpha(10 ** 6, h) - (1 - h)) < 1e-15
        # before saturation it is the running-mean weight 1/(n+1)
        assert oracle.blend_alpha(0, h) == 1.0
        assert oracle.blend_alpha(nmax - 1, h) == 1.0 / nmax
    # the prose reading (N_max-1)/N_max would print 0.90 for N_max=10, not 0.91
    assert round(9 / 10, 2) != 0.91


def _sky_scene(value, dims=(1, 1, 1)):
    return scenes.Scene(
        name="sky", positions=np.zeros((0, 3), np.float32), indices=np.zeros((0, 3), np.int32),
        albedo=np.zeros((0, 3), np.float32), light_a=np.zeros((0, 3), np.float32),
        light_b=np.zeros((0, 3), np.float32), light_intensity=np.zeros((0, 3), np.float32),
        sky=np.array(value, np.float32), grid_origin=np.zeros(3, np.float32),
        grid_spacing=np.ones(3, np.float32), grid_dims=np.array(dims, np.int32), frames=2)


def test_pin6_running_mean_then_step_response():
    # Cornell room, 1 frame, <=33 samples per texel from empty: exact mean.
    vol = oracle.OracleVolume(scenes.cornell(), seed=3)
    out = vol.update(0, adaptive=False, n_uniform=200, keep_rays=True)
    for q in (0, 21, 42, 63):
        b = out["ray_base"][q]
        bins = out["irr_bin"][b:b + 200]
        rgb = out["rays"][b:b + 200, :3]
        for k in range(36):
            sel = bins == k
            if 0 < sel.sum() <= 33:
                assert np.allclose(vol.irr[q].reshape(36, 3)[k], rgb[sel].mean(axis=0),
                                   rtol=1e-12, atol=1e-15)
    # saturated step response: after a texel has >= 34 samples of 0, switch
    # the sky to 1; after k more samples the texel holds 1 - h^k.
    vol = oracle.OracleVolume(_sky_scene([0.0, 0.0, 0.0]), seed=1)
    for f in range(6):
        vol.update(f, adaptive=False, n_uniform=400)
    assert vol.irr_n.min() >= 34
    n0 = vol.irr_n.copy().astype(np.int64)
    vol.sc.sky = np.ones(3, np.float32)
    out = vol.update(6, adaptive=False, n_uniform=400, keep_rays=True)
    k = np.bincount(out["irr_bin"], minlength=36)
    expect = 1.0 - vol.h ** k
    assert np.allclose(vol.irr.reshape(36, 3)[:, 0], expect, rtol=1e-12)
    assert np.array_equal(vol.irr_n[0], np.minimum(n0[0] + k, 255))


def test_fp16_rounding_is_rne():
    # exactly representable values are unchanged; halfway cases go to even
    assert oracle.round_half(1.0) == 1.0
    assert oracle.round_half(1.0 + 2 ** -11) == 1.0          # halfway, to even (1.0)
    assert oracle.round_half(1.0 + 3 * 2 ** -11) == 1.0 + 2 ** -9  # halfway, to even
    assert oracle.round_half(65504.0) == 65504.0
    assert math.isinf(oracle.round_half(65520.0))
    assert oracle.round_half(2 ** -25) == 0.0                 # halfway to 0 (even)
    assert oracle.round_half(3 * 2 ** -25) == 2 ** -23
    rng = np.random.default_rng(0)
    x = rng.uniform(-100, 100, 5000)
    ref = x.astype(np.float16).astype(np.float64)  # numpy converts directly with RNE
    assert np.array_equal(np.array([oracle.round_half(v) for v in x]), ref)


# --------------------------------------------------------- O5: detection

def _grid(dims):
    return oracle.make_grid(np.zeros(3, np.float32), np.ones(3, np.float32),
                            np.array(dims, np.int32))


def _detect_run(dims, frames_q, theta=8, mu=2):
    import ctypes as C
    L = oracle.lib()
    g = _grid(dims)
    P = int(np.prod(dims))
    st = dict(qvp=np.zeros(P * 8, np.uint16), qrp=np.zeros(P * 8, np.uint16),
              tv=np.zeros(P * 8, np.int32), tr=np.zeros(P * 8, np.int32),
              s=np.zeros(P, np.int64))
    scores = []
    for f, (qv, qr) in enumerate(frames_q):
        qv = np.ascontiguousarray(qv, np.uint16)
        qr = np.ascontiguousarray(qr, np.uint16)
        L.orc_detect(C.byref(g), f, theta, mu, oracle._p(qv), oracle._p(qr), oracle._p(st["qvp"]),
                     oracle._p(st["qrp"]), oracle._p(st["tv"]), oracle._p(st["tr"]),
                     oracle._p(st["s"]))
        scores.append(st["s"].copy())
    return scores, st


def test_pin7_static_scene_scores_zero():
    rng = np.random.default_rng(0)
    dims = (5, 3, 4)
    P = 60
    q = (rng.integers(0, 1024, P * 8), rng.integers(0, 1024, P * 8))
    scores, _ = _detect_run(dims, [q, q, q, q])
    assert all(np.all(s == 0) for s in scores)
    n, off, _ = oracle.allocate(scores[-1], 64 * P + 17, 8, 512)
    assert np.all(n[:17] == 65) and np.all(n[17:] == 64)


def test_pin7_box_sum_identity_and_locality():
    rng = np.random.default_rng(1)
    dims = (7, 6, 9)
    P = int(np.prod(dims))
    qv0 = rng.integers(0, 1024, P * 8)
    qr0 = rng.integers(0, 1024, P * 8)
    qr1 = rng.integers(0, 1024, P * 8)
    ones = np.ones(P * 8)
    scores, st = _detect_run(dims, [(qv0, qr0), (ones, qr1)], mu=3)
    tv, tr = st["tv"].astype(np.int64), st["tr"].astype(np.int64)
    assert np.array_equal(tv, np.abs(1 - qv0)) and np.array_equal(tr, np.abs(qr1 - qr0))
    # sum_i score_i = sum_j (Tv_j + mu Tr_j) * #{grid probes in the 5x5x5 box at j}
    def span(x, D):
        return min(x + 2, D - 1) - max(x - 2, 0) + 1
    mult = np.zeros(P, np.int64)
    for z in range(dims[2]):
        for y in range(dims[1]):
            for x in range(dims[0]):
                mult[x + dims[0] * (y + dims[1] * z)] = span(x, dims[0]) * span(y, dims[1]) * span(z, dims[2])
    rhs = ((tv + 3 * tr).reshape(P, 8).sum(axis=1) * mult).sum()
    assert scores[1].sum() == rhs
    # a single pulse reaches exactly the 5x5x5 neighbourhood
    dims = (9, 9, 9)
    P = 729
    z0 = np.zeros(P * 8)
    qv = np.full(P * 8, 3)
    pulse = z0.copy()
    c = 4 + 9 * (4 + 9 * 4)
    pulse[c * 8 + 5] = 100
    scores, _ = _detect_run(dims, [(qv, z0), (qv, pulse)])
    s = scores[1].reshape(9, 9, 9)
    assert np.all(s[2:7, 2:7, 2:7] == 3 * 2 * 100)
    s[2:7, 2:7, 2:7] = 0
    assert np.all(s == 0)


def test_pin7_trigger_decays_to_zero():
    dims = (1, 1, 1)
    z = np.zeros(8)
    pulse = np.zeros(8)
    pulse[0] = 1023
    qv = np.ones(8)
    frames = [(qv, z), (qv, pulse)] + [(qv, pulse)] * 30
    scores, _ = _detect_run(dims, frames, theta=8)
    odd = [s[0] for f, s in enumerate(scores) if f % 2 == 1]
    delta = math.ceil(1023 / 8)
    # T = 1023, 1023-d, ... then 0 after ceil(1023/delta) = 8 detection steps
    assert odd[0] == 2 * 1023
    assert odd[1:9] == [2 * max(0, 1023 - k * delta) for k in range(1, 9)]
    assert odd[8] == 0 and all(v == 0 for v in odd[8:])


def test_pin7_light_switched_on_changes_only_lit_pilots():
    sc = scenes.cornell()
    sc.light_intensity = np.zeros((1, 3), np.float32)
    vol = oracle.OracleVolume(sc, seed=2)
    vol.set_frame_inputs(0)
    qv0, qr0 = vol.pilots(0)
    assert np.all(qr0 == 0)
    vol.sc.light_intensity = np.full((1, 3), 5.0, np.float32)
    vol.set_frame_inputs(1)
    qv1, qr1 = vol.pilots(1)
    assert np.array_equal(qv0, qv1)  # same directions within a pair, static geometry
    changed = qr1 != qr0
    assert changed.any()
    score = vol.detect(0, qv0, qr0)
    score = vol.detect(1, qv1, qr1)
    assert np.all(vol.tv == 0) and np.array_equal(vol.tr > 0, changed)



# ---- pilot codes (eq. ProbeVis; Sec. 4.1.3; App. B round-down), O5

def _pilot_plane_scene(H_lo, rho, I, light_h, sky, half=1.0e4):
    """Ground quad z = 0 (normal +z) under a probe grid whose layers sit at
    heights H_lo + k*0.45; one point light at (0.3, -0.2, light_h)."""
    pos, idx = _quad(-half, half, -half, half, 0.0)
    return scenes.Scene(
        name="pilot_plane", positions=pos, indices=idx, albedo=np.full((2, 3), rho, np.float32),
        light_a=np.array([[0.3, -0.2, light_h]], np.float32),
        light_b=np.array([[0.3, -0.2, light_h]], np.float32),
        light_intensity=np.array([I], np.float32), sky=np.array(sky, np.float32),
        grid_origin=np.array([0.1, -0.35, H_lo], np.float32),
        grid_spacing=np.array([0.5, 0.7, 0.45], np.float32),
        grid_dims=np.array([2, 3, 3], np.int32), frames=2)


def _pilot_expect(sc, seed, frame, beta=5.0):
    """Pilot codes written out from the geometry: a downward pilot of probe
    p meets z = 0 at t = p_z/|d_z| and lands at x = p + t d; an upward one
    leaves the scene. Qv = min(1023, floor(1024 exp(-2t/s))), 0 on a miss;
    Qr = min(1023, floor(1024 min(lum, beta)/beta)) with Rec. 709 luminance
    of (rho/pi) I cos/|l|^2 at x (l = light - x) or of the sky on a miss.
    Also returns the distance of 1024 f to the nearest integer (code edges)."""
    dims = sc.grid_dims.astype(np.int64)
    org = sc.grid_origin.astype(np.float64)
    spc = sc.grid_spacing.astype(np.float64)
    s = float(np.sqrt(np.sum(spc * spc)))
    rho = sc.albedo[0].astype(np.float64)
    I = sc.light_intensity[0].astype(np.float64)
    lp = sc.light_positions(frame)[0].astype(np.float64)
    sky = sc.sky.astype(np.float64)
    w709 = np.array([0.2126, 0.7152, 0.0722])
    P = int(np.prod(dims))
    qv = np.zeros(P * 8, np.int64)
    qr = np.zeros(P * 8, np.int64)
    edge = np.full(P * 8, np.inf)
    for i in range(P):
        x_, y_, z_ = i % dims[0], (i // dims[0]) % dims[1], i // (dims[0] * dims[1])
        p = org + np.array([x_, y_, z_]) * spc
        for k in range(8):
            d = oracle.pilot_dir(seed, i, k, frame // 2)
            if d[2] < 0.0:
                t = p[2] / -d[2]
                x = p + t * d
                fv = 1024.0 * math.exp(-2.0 * t / s)
                ell = lp - x
                dist = float(np.linalg.norm(ell))
                L = rho / math.pi * I * max(0.0, ell[2] / dist) / (dist * dist)
            else:
                fv = 0.0
                L = sky
            fr = 1024.0 * min(float(w709 @ L), beta) / beta
            qv[8 * i + k] = min(1023, math.floor(fv))
            qr[8 * i + k] = min(1023, math.floor(fr))
            for f_ in (fv, fr):
                if 0.5 < f_ < 1023.0:
                    edge[8 * i + k] = min(edge[8 * i + k], abs(f_ - round(f_)))
    return qv, qr, edge


@pytest.mark.parametrize("channel", [0, 1, 2])
def test_pilot_codes_over_a_lit_plane(channel):
    """Known hit distances and a known lit Lambertian plane give the codes
    of eq. ProbeVis (exp(-2t/s), not exp(-t/s)) and of the radiance term
    (Rec. 709 weights, one colour channel at a time so that each weight is
    checked on its own; a coloured sky for the upward pilots); misses give
    Qv = 0. Codes within 1e-6 of an integer edge are skipped."""
    I = [0.0, 0.0, 0.0]
    I[channel] = 2.5
    sky = [0.5, 1.0, 2.0]
    sc = _pilot_plane_scene(0.2, (0.9, 0.6, 0.8), I, light_h=2.0, sky=sky)
    for frame in (0, 1, 2):
        vol = oracle.OracleVolume(sc, seed=31 + channel, use_bvh=False)
        vol.set_frame_inputs(frame)
        qv, qr = vol.pilots(frame)
        eqv, eqr, edge = _pilot_expect(sc, 31 + channel, frame)
        ok = edge > 1e-6
        assert ok.mean() > 0.98
        assert np.array_equal(qv[ok], eqv[ok]), np.nonzero(qv[ok] != eqv[ok])
        assert np.array_equal(qr[ok], eqr[ok]), np.nonzero(qr[ok] != eqr[ok])
        down = np.array([oracle.pilot_dir(31 + channel, r // 8, r % 8, frame // 2)[2] < 0
                         for r in range(qv.size)])
        assert np.all(qv[~down] == 0) and np.mean(qv[down] > 0) > 0.5
        # the sky's luminance 0.9659... gives floor(1024 * 0.9659 / 5) = 197 on every miss
        assert np.all(qr[~down] == 197)
        # some lit pilots carry a non-zero radiance code
        assert np.count_nonzero(qr[down]) > 0


def test_pilot_radiance_code_clamps_at_beta():
    """Luminance at or above beta saturates the radiance code at 1023; a
    black sky gives 0 on every miss."""
    sc = _pilot_plane_scene(0.2, (0.9, 0.9, 0.9), [4000.0, 4000.0, 4000.0], light_h=2.0,
                            sky=[0.0, 0.0, 0.0])
    vol = oracle.OracleVolume(sc, seed=77, use_bvh=False)
    vol.set_frame_inputs(0)
    qv, qr = vol.pilots(0)
    eqv, eqr, edge = _pilot_expect(sc, 77, 0)
    down = np.array([oracle.pilot_dir(77, r // 8, r % 8, 0)[2] < 0 for r in range(qv.size)])
    assert np.mean(eqr[down] == 1023) > 0.5  # lum >= beta near the light
    ok = edge > 1e-6
    assert np.array_equal(qr[ok], eqr[ok])
    assert np.all(qr[~down] == 0)
    assert np.array_equal(qv[ok], eqv[ok])


def test_pilot_code_at_distance_zero_saturates():
    """A pilot that leaves a probe lying on a surface has t -> 0 and
    1024 exp(0) = 1024, clamped to the 10-bit maximum 1023; codes are
    monotone in distance."""
    sc = _pilot_plane_scene(1e-7, (0.5, 0.5, 0.5), [0.0, 0.0, 0.0], light_h=2.0, sky=[0, 0, 0])
    vol = oracle.OracleVolume(sc, seed=5, use_bvh=False)
    vol.set_frame_inputs(0)
    qv, _ = vol.pilots(0)
    dims = sc.grid_dims
    lowest = [i for i in range(int(np.prod(dims))) if i // (dims[0] * dims[1]) == 0]
    for i in lowest:
        for k in range(4, 8):  # octants with bit 2 set point down (-z)
            d = oracle.pilot_dir(5, i, k, 0)
            if -d[2] > 1e-3:
                assert qv[8 * i + k] == 1023
    # probes higher up see the plane further away: lower codes on average
    per_layer = [np.mean([qv[8 * i + k] for i in range(int(np.prod(dims)))
                          if i // (dims[0] * dims[1]) == z for k in range(4, 8)]) for z in range(3)]
    assert per_layer[0] > per_layer[1] > per_layer[2]


def test_pilot_reuse_adds_the_pilot_samples_on_the_first_frame_of_a_pair():
    """Pilot reuse (Sec. 4.4): on the first frame of each pilot pair every
    probe's 8 pilot samples also enter its caches, each into the texels of its
    own direction; on the second frame (same directions) they do not. Over a
    lit plane the pilot records equal the closed form, and after the first
    frame every sampled texel holds the exact mean of its samples (pilots and
    probe rays, at most 33 of them, so the moving average is a running mean)."""
    sc = _pilot_plane_scene(0.2, (0.9, 0.6, 0.8), [2.5, 1.5, 0.5], light_h=2.0, sky=[0.5, 1.0, 2.0])
    P = sc.num_probes
    seed = 41
    kw = dict(adaptive=True, budget=P * 16, n_min=16, n_max=16, keep_rays=True)
    vol = oracle.OracleVolume(sc, seed=seed, use_bvh=False)
    plain = oracle.OracleVolume(sc, seed=seed, use_bvh=False)
    out = vol.update(0, pilot_reuse=True, **kw)
    plain.update(0, **kw)
    # pilot records against the plane's closed form
    org = sc.grid_origin.astype(np.float64)
    spc = sc.grid_spacing.astype(np.float64)
    dims = sc.grid_dims
    rho = sc.albedo[0].astype(np.float64)
    I = sc.light_intensity[0].astype(np.float64)
    lp = sc.light_positions(0)[0].astype(np.float64)
    pdirs = np.zeros((P, 8, 3))
    for i in range(P):
        p = org + np.array([i % dims[0], (i // dims[0]) % dims[1], i // (dims[0] * dims[1])]) * spc
        for k in range(8):
            d = oracle.pilot_dir(seed, i, k, 0)
            pdirs[i, k] = d
            r = 8 * i + k
            if d[2] < 0:
                t = p[2] / -d[2]
                x = p + t * d
                ell = lp - x
                dist = np.linalg.norm(ell)
                L = rho / math.pi * I * max(0.0, ell[2] / dist) / dist ** 2
                assert abs(out["pilot_t"][r] - t) <= 1e-12 * t
            else:
                L = sc.sky.astype(np.float64)
                assert np.isinf(out["pilot_t"][r])
            assert np.allclose(out["pilot_rgb"][r], L, rtol=1e-12, atol=0)
    # counts: the probe rays' bins plus the pilots' bins
    for q in range(P):
        b = out["ray_base"][q]
        ib = out["irr_bin"][b:b + 16]
        pib = np.array([oracle.oct_bin(pdirs[q, k], 6)[0] for k in range(8)])
        exp_n = np.bincount(np.concatenate([ib, pib]), minlength=36)
        assert np.array_equal(vol.irr_n[q], exp_n)
        assert np.array_equal(plain.irr_n[q], np.bincount(ib, minlength=36))
        # each sampled texel: the mean of its samples
        rgb = np.concatenate([out["rays"][b:b + 16, :3], out["pilot_rgb"][8 * q:8 * q + 8]])
        bins = np.concatenate([ib, pib])
        irr = vol.irr[q].reshape(36, 3)
        for k in np.nonzero(exp_n)[0]:
            assert np.allclose(irr[k], rgb[bins == k].mean(axis=0), rtol=1e-12, atol=1e-15)
    # second frame of the pair: the same pilot directions, not reused again
    n0 = vol.irr_n.copy()
    out1 = vol.update(1, pilot_reuse=True, **kw)
    for q in range(P):
        b = out1["ray_base"][q]
        inc = np.bincount(out1["irr_bin"][b:b + 16], minlength=36)
        assert np.array_equal(vol.irr_n[q].astype(int) - n0[q], inc)

# -------------------------------------------------------- O6: allocation

def _brute_lambda(w, E, Bp):
    """lambda* by scanning every breakpoint of the step function."""
    cands = {0, 1 << 31}
    for wi in w:
        if wi == 0:
            continue
        for m in range(1, E + 1):
            lam = -(-(m << 32) // wi)  # ceil(m*2^32 / w)
            if lam <= (1 << 31):
                cands.add(lam)
    best = 0
    for lam in sorted(cands):
        tot = sum(min(E, (lam * wi) >> 32) for wi in w)
        if tot <= Bp:
            best = max(best, lam)
    # lambda* is the last integer before the next breakpoint that overflows
    nxt = [c for c in sorted(cands) if c > best]
    for c in nxt:
        tot = sum(min(E, (c * wi) >> 32) for wi in w)
        if tot > Bp:
            return c - 1
        best = c
    return 1 << 31


def _weights(score):
    mx = int(max(score))
    if mx == 0:
        return [1 << 31] * len(score)
    b = mx.bit_length()
    return [(int(s) << (32 - b)) if b <= 32 else (int(s) >> (b - 32)) for s in score]


def test_pin8_allocation_matches_breakpoint_scan():
    rng = np.random.default_rng(4)
    for trial in range(60):
        P = int(rng.integers(1, 9))
        n_min = int(rng.integers(1, 5))
        n_max = n_min + int(rng.integers(0, 12))
        score = rng.integers(0, 3000, P)
        if trial % 7 == 0:
            score[:] = 0
        if trial % 11 == 0:
            score = rng.integers(0, 2 ** 40, P)
        budget = P * n_min + int(rng.integers(0, P * (n_max - n_min) + 3))
        n, off, lam = oracle.allocate(score, budget, n_min, n_max)
        w = _weights(score)
        E = n_max - n_min
        Bp = budget - P * n_min
        assert lam == _brute_lambda(w, E, Bp)
        e0 = [min(E, (lam * wi) >> 32) for wi in w]
        R = Bp - sum(e0)
        bonus = [0] * P
        for i in range(P):
            if R > 0 and min(E, ((lam + 1) * w[i]) >> 32) > e0[i]:
                bonus[i] = 1
                R -= 1
        assert list(n) == [n_min + e0[i] + bonus[i] for i in range(P)]
        assert np.all(n >= n_min) and np.all(n <= n_max)
        assert off[0] == 0 and np.array_equal(np.diff(off), n)
        if sum(min(E, (((1 << 31) + 1) * wi) >> 32) for wi in w) > Bp:
            assert n.sum() == budget  # not saturated: the budget is spent exactly


def test_pin8_allocation_properties():
    rng = np.random.default_rng(5)
    P = 2048
    score = rng.integers(0, 10 ** 6, P)
    B = 2 ** 19
    n, off, lam = oracle.allocate(score, B, 32, 1024)
    assert n.sum() == B and n.min() >= 32 and n.max() <= 1024
    # monotone in a score while the normalisation shift is unchanged
    i = int(np.argmin(score))
    s2 = score.copy()
    s2[i] += 1000
    n2, _, _ = oracle.allocate(s2, B, 32, 1024)
    assert n2[i] >= n[i]
    # all-zero scores: uniform, remainder to the lowest indices
    n3, _, _ = oracle.allocate(np.zeros(P, np.int64), B + 5, 32, 1024)
    assert np.all(n3[:5] == 257) and np.all(n3[5:] == 256)
    with pytest.raises(ValueError):
        oracle.allocate(score, 32 * P - 1, 32, 1024)


# ---------------------------------------------------------------- packed texels
# The packed words of eq. rgbEnc / App. B (R9 G9 B8 + N6; two 13-bit depth
# channels + N6): binary32 moving averages, exact codes, decoded values
# rounded once to binary32. Pins: every code boundary and every decoded value
# of the four channel types against 50-digit arithmetic, the closed form of
# the encoding, the round-down property the paper states for its
# quantisation (dark samples drive a texel to zero), the fixed point of the
# quantised moving average, and the count field.

PACK_CHANNELS = [(5.0, 15.0, 9), (5.0, 15.0, 8), (5.0, 15.0, 13), (8.0, 20.0, 13)]


def _f32_up(f):
    return np.nextafter(np.float32(f), np.float32(np.inf))


def _f32_down(f):
    return np.nextafter(np.float32(f), np.float32(0.0))


@pytest.mark.parametrize("beta,gamma,bits", PACK_CHANNELS)
def test_packed_codes_exact_at_every_boundary(beta, gamma, bits):
    """Code k begins at t_k = (e^(beta k / qmax) - 1) / gamma. For every k the
    binary32 value just above t_k encodes to k and the one just below to
    k - 1, and both lie farther from the boundary (in code units, 50-digit
    arithmetic) than any FP64 rounding could reach; so the encoder is the
    exact floor for every binary32 input."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    qmax = (1 << bits) - 1
    B, G = Decimal(beta), Decimal(gamma)
    min_margin = Decimal(1)
    for k in range(1, qmax + 1):
        t = ((B * k / qmax).exp() - 1) / G
        f = np.float32(float(t))
        while Decimal(float(f)) < t:
            f = _f32_up(f)
        while Decimal(float(_f32_down(f))) >= t:
            f = _f32_down(f)
        lo = _f32_down(f)
        assert oracle.pack_encode(float(f), beta, gamma, bits) == k, (k, float(f))
        assert oracle.pack_encode(float(lo), beta, gamma, bits) == k - 1, (k, float(lo))
        for x, side in ((f, 1), (lo, -1)):
            u = (G * Decimal(float(x)) + 1).ln() / B * qmax
            min_margin = min(min_margin, side * (u - k))
    # FP64 evaluation errs by a few ulps of log1p (<= 5) scaled by qmax / beta
    # (<= 1639) plus the rounding of the product: below 5e-12 code units;
    # the nearest binary32 input to any boundary is 3.7e-10 away (13 bits)
    assert min_margin > Decimal("1e-10"), min_margin
    # saturation: everything at or above t_qmax is qmax
    assert oracle.pack_encode(3.0e38, beta, gamma, bits) == qmax
    assert oracle.pack_encode(0.0, beta, gamma, bits) == 0
    assert oracle.pack_encode(-1.0, beta, gamma, bits) == 0


@pytest.mark.parametrize("beta,gamma,bits", PACK_CHANNELS)
def test_packed_decode_is_the_rounded_exact_value(beta, gamma, bits):
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    qmax = (1 << bits) - 1
    B, G = Decimal(beta), Decimal(gamma)
    for q in range(qmax + 1):
        d = ((B * q / qmax).exp() - 1) / G
        f = np.float32(float(d))
        cands = [_f32_down(f), f, _f32_up(f)]
        best = min(cands, key=lambda c: (abs(Decimal(float(c)) - d), int(np.float32(c).view(np.uint32)) & 1))
        assert oracle.pack_decode(q, beta, gamma, bits) == float(best), (q, float(best))


@pytest.mark.parametrize("beta,gamma,bits", PACK_CHANNELS)
def test_packed_encode_closed_form(beta, gamma, bits):
    qmax = (1 << bits) - 1
    rng = np.random.default_rng(bits)
    vs = np.concatenate([np.exp(rng.uniform(-12, 4, 3000)), [0.0, 1e-30]]).astype(np.float32)
    vmax = (math.exp(beta) - 1.0) / gamma
    for v in vs:
        q = oracle.pack_encode(float(v), beta, gamma, bits)
        exact = min(math.log(gamma * float(v) + 1.0), beta) / beta * qmax
        if abs(exact - round(exact)) > 1e-4 * max(1.0, exact):  # not on a code boundary
            assert q == min(math.floor(exact), qmax), (v, q, exact)
        d = oracle.pack_decode(q, beta, gamma, bits)
        # round down: the stored value never exceeds the sample ...
        assert d <= float(v) * (1 + 1e-6) + 1e-12
        # ... and lies within one code of it (unless saturated)
        if q < qmax:
            assert float(v) <= oracle.pack_decode(q + 1, beta, gamma, bits) * (1 + 1e-6)
        else:
            assert float(v) >= vmax * (1 - 1e-5)
    assert oracle.pack_decode(0, beta, gamma, bits) == 0.0
    assert abs(oracle.pack_decode(qmax, beta, gamma, bits) - vmax) <= 1e-6 * vmax
    dec = [oracle.pack_decode(q, beta, gamma, bits) for q in range(0, qmax + 1, max(1, qmax // 511))]
    assert all(b > a for a, b in zip(dec, dec[1:]))


def _blend_one_texel(samples, h=0.97, start_word=0):
    """Feed a sample sequence to one irradiance texel and one depth texel."""
    m = len(samples)
    rec = np.zeros((max(m, 1), 4), np.float32)
    rec[:m, 0] = rec[:m, 1] = rec[:m, 2] = samples
    rec[:m, 3] = samples
    irr = np.full(36, start_word, np.uint32)
    dep = np.full(196, start_word, np.uint32)
    zeros = np.zeros(max(m, 1), np.uint16)
    oracle.packed_blend([m], [0], rec, zeros, zeros, 6, 14, 1.0, oracle.TAU_MAX,
                        oracle.packed_alpha_table(h), irr, dep)
    return irr, dep


def test_packed_dark_samples_reach_zero():
    # the paper's reason for round-down: low samples pull a texel to zero
    full = (511 | (511 << 9) | (255 << 18) | (63 << 26))
    irr, _ = _blend_one_texel(np.zeros(4000, np.float32), start_word=full)
    assert irr[0] & 0x3FFFFFF == 0 and irr[0] >> 26 == 63


def test_packed_constant_input_fixed_point_and_count():
    h = 0.97
    for x in (0.02, 0.3, 1.0, 4.0):
        for m in (1, 5, 40, 600):
            irr, dep = _blend_one_texel(np.full(m, x, np.float32), h)
            assert irr[0] >> 26 == min(m, 63) and dep[0] >> 26 == min(m, 63)
            assert np.all(irr[1:] == 0) and np.all(dep[1:] == 0)
            vals, _ = oracle.unpack_words(irr[:1], oracle.PACK_IRR)
            q = int(irr[0] & 0x1FF)
            d, d_next = vals[0, 0], oracle.pack_decode(q + 1, 5.0, 15.0, 9)
            assert d <= x * (1 + 1e-6)
            if m == 1:
                assert q == oracle.pack_encode(x, 5.0, 15.0, 9)  # first sample: weight 1
            else:
                # a fixed point of the quantised average lies below x by less
                # than one code step divided by the step weight
                a = max(1.0 / min(m, 63), 1.0 - h)
                assert x - d <= (d_next - d) / a * (1 + 1e-5)


# ------------------------------------------------------- Metropolis chains
# The static chain (Alg. MarkovChainMT with Alg. MetropolisStep, target
# h = exp(min(g/f, 1)) f of Sec. 4.8). Pins: the properties of h the paper
# states (g is trusted only where f is low: h in [f, e f], h = f without
# feedback, h = e f once g >= f, zero where f is zero), and the theorem that
# makes the sampler correct: a symmetric random walk with Metropolis
# acceptance and rejection outside the domain has h (restricted to the domain)
# as its stationary density. Probe cells and octants are given different f;
# the chains' occupancy must match their h-weighted volumes.

def _chain_grid(dims=(2, 2, 2)):
    return oracle.make_grid(np.zeros(3, np.float32), np.ones(3, np.float32),
                            np.asarray(dims, np.int32))


def test_chain_target_properties():
    g = _chain_grid()
    P, r = 8, 6
    rng = np.random.default_rng(3)
    qv = rng.integers(1, 1024, P * 8).astype(np.uint16)
    qv[8 * 3 + 5] = 0
    for gval in (0.0, 0.05, 0.3, 2.0):
        irr = np.full((P, r * r * 3), gval)
        for _ in range(200):
            x = np.concatenate([rng.uniform(0, 1, 3), rng.uniform(-1, 1, 2)])
            h, pr, tie = oracle.chain_h(g, qv, irr, r, x)
            d = np.zeros(3)
            oracle.lib().orc_chain_dir(oracle._p(np.ascontiguousarray(x[3:])), oracle._p(d))
            k = int(d[0] < 0) | int(d[1] < 0) << 1 | int(d[2] < 0) << 2
            assert pr == int(np.round(x[0])) + 2 * (int(np.round(x[1])) + 2 * int(np.round(x[2])))
            f = qv[8 * pr + k] / 1024.0
            if f == 0:
                assert h == 0.0
                continue
            assert f * (1 - 1e-12) <= h <= math.e * f * (1 + 1e-12)
            if gval == 0.0:
                assert abs(h - f) <= 1e-12
            if gval >= f:
                assert abs(h - math.e * f) <= 1e-12 * h


def _octant_of_uv(uv):
    # signs of the decoded direction: x follows u, y follows v, z < 0 outside
    # the diamond |u| + |v| <= 1
    u, v = uv[:, 0], uv[:, 1]
    return (u < 0).astype(int) | (v < 0).astype(int) << 1 | (np.abs(u) + np.abs(v) > 1).astype(int) << 2


def test_chain_stationary_distribution():
    g = _chain_grid()
    P, r = 8, 6
    rng = np.random.default_rng(11)
    qv = rng.integers(64, 1024, P * 8).astype(np.uint16)
    irr = np.zeros((P, r * r * 3))
    irr[2] = 0.4  # one probe with feedback: h = exp(min(0.4/f, 1)) f there
    cp = oracle.ChainParams(1024, 64, 0, 0.3, 0.35)
    state = np.zeros((1024, 5))
    occ = np.zeros(P * 8)
    for frame in range(96):
        out = oracle.chain_frame(g, cp, 99, frame, qv, irr, r, state, init=(frame == 0))
        if frame < 2:
            continue  # burn-in across frames
        cell = 8 * out["sample_probe"] + _octant_of_uv(out["sample_uv"])
        occ += np.bincount(cell, minlength=P * 8)
    # h is constant on each (probe cell, octant); the cells have equal volume
    # in this 2x2x2 grid and the octants equal areas in the octahedral square
    f = qv / 1024.0
    gl = np.zeros(P * 8)
    gl[16:24] = 0.4
    h = np.exp(np.minimum(gl / f, 1.0)) * f
    want = h / h.sum()
    got = occ / occ.sum()
    assert np.max(np.abs(got - want) / want) < 0.06, np.max(np.abs(got - want) / want)
    # a sampler that ignored h would be uniform: far from the target
    assert np.max(np.abs(1.0 / (P * 8) - want) / want) > 0.5


def test_chain_samples_layout_and_domain():
    g = _chain_grid((3, 2, 4))
    P, r = 24, 6
    qv = np.full(P * 8, 500, np.uint16)
    irr = np.zeros((P, r * r * 3))
    cp = oracle.ChainParams(16, 10, 3, 1.0, 0.2)
    state = np.zeros((16, 5))
    a = oracle.chain_frame(g, cp, 5, 0, qv, irr, r, state, init=True)
    assert len(a["sample_probe"]) == 16 * 6 and len(a["accept"]) == 16 * 10
    assert np.all(state[:, 0] >= 0) and np.all(state[:, 0] <= 2) and np.all(state[:, 2] <= 3)
    assert np.all(np.abs(state[:, 3:]) <= 1)
    # the last sample of a chain is its final state
    uv_last = a["sample_uv"].reshape(16, 6, 2)[:, -1]
    assert np.array_equal(uv_last, state[:, 3:])
    # deterministic in the seed, different across seeds
    s2 = np.zeros((16, 5))
    b = oracle.chain_frame(g, cp, 5, 0, qv, irr, r, s2, init=True)
    assert np.array_equal(a["sample_uv"], b["sample_uv"]) and np.array_equal(state, s2)
    s3 = np.zeros((16, 5))
    c = oracle.chain_frame(g, cp, 6, 0, qv, irr, r, s3, init=True)
    assert not np.array_equal(a["sample_uv"], c["sample_uv"])


def _np_oct_uv(d):
    """Octahedral coordinates of unit directions (Cigolle et al. 2014), numpy."""
    d = np.asarray(d, np.float64)
    p = d[:, :2] / np.abs(d).sum(axis=1, keepdims=True)
    low = d[:, 2] < 0
    s = np.where(p >= 0, 1.0, -1.0)
    fold = (1.0 - np.abs(p[:, ::-1])) * s
    return np.where(low[:, None], fold, p)


def _np_oct_dir(uv):
    uv = np.asarray(uv, np.float64)
    z = 1.0 - np.abs(uv).sum(axis=1)
    s = np.where(uv >= 0, 1.0, -1.0)
    xy = np.where((z < 0)[:, None], (1.0 - np.abs(uv[:, ::-1])) * s, uv)
    d = np.concatenate([xy, z[:, None]], axis=1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_chain_update_two_rays_per_sample():
    """A chain frame on a fresh volume with hysteresis 0: each sample adds one
    irradiance count in the texel of d(uv) and one depth count in the texel of
    -d at its nearest probe, and each depth texel then holds tau of the last
    such sample's -d ray, found here by brute force over the triangles."""
    sc = scenes.cornell()
    ora = oracle.OracleVolume(sc, seed=21, hysteresis=0.0)
    cp = oracle.ChainParams(24, 12, 3, 0.5, oracle.SIGMA_DIR)
    state = np.zeros((24, 5))
    out = ora.chain_update(0, cp, state, init=True)
    ri, rd = ora.irr_res - 2, ora.depth_res - 2
    perm, sp, suv = out["perm"], out["sample_probe"], out["sample_uv"]
    assert len(sp) == 24 * 8 and out["n"].sum() == len(sp)
    assert np.array_equal(np.sort(sp, kind="stable"), sp[perm])
    d = _np_oct_dir(suv[perm])
    probes = sp[perm]
    bi = np.clip(np.floor((_np_oct_uv(d) + 1.0) * 0.5 * ri).astype(int), 0, ri - 1)
    bd = np.clip(np.floor((_np_oct_uv(-d) + 1.0) * 0.5 * rd).astype(int), 0, rd - 1)
    ki = bi[:, 1] * ri + bi[:, 0]
    kd = bd[:, 1] * rd + bd[:, 0]
    want_i = np.zeros((ora.P, ri * ri), np.int64)
    want_d = np.zeros((ora.P, rd * rd), np.int64)
    np.add.at(want_i, (probes, ki), 1)
    np.add.at(want_d, (probes, kd), 1)
    assert np.array_equal(ora.irr_n, want_i) and np.array_equal(ora.dep_n, want_d)
    s = float(np.sqrt(np.sum(np.asarray(sc.grid_spacing, np.float64) ** 2)))
    last = {}
    for k in range(len(probes)):
        last[(probes[k], kd[k])] = k
    for (p, b), k in last.items():
        dx, dy, _ = (int(x) for x in sc.grid_dims)
        o = np.asarray(sc.grid_origin, np.float64) + np.asarray(sc.grid_spacing, np.float64) * \
            np.array([p % dx, (p // dx) % dy, p // (dx * dy)])
        h = ora.scene.closest_hit(o, -d[k], brute=True)
        tau = min(h.t / s, ora.tau_max) if h.tri >= 0 else ora.tau_max
        assert abs(ora.dep[p, 2 * b] - tau) <= 1e-9 * max(tau, 1.0), (p, b)
        assert abs(ora.dep[p, 2 * b + 1] - tau * tau) <= 1e-9 * max(tau * tau, 1.0), (p, b)


# ---- dynamic chains on 3x3x3 virtual proxies (Sec. 4.9)

@pytest.mark.parametrize("r", [5, 6, 7, 14])
def test_octant_texels_partition_the_map(r):
    """The octants' texel-centre lists partition the r x r map, and each
    centre's direction lies in its octant (sign of x, y, z; centres on the
    diagonal |u| + |v| = 1 give z = 0 and belong to the upper half)."""
    seen = np.zeros(r * r, np.int64)
    for k in range(8):
        lst = oracle.octant_texels(r, k)
        seen[lst] += 1
        for t in lst:
            d = oracle.texel_centre_dir(r, int(t))
            assert abs(np.linalg.norm(d) - 1.0) < 1e-12
            if abs(d[0]) > 1e-12:
                assert (d[0] < 0) == bool(k & 1)
            if abs(d[1]) > 1e-12:
                assert (d[1] < 0) == bool(k & 2)
            if abs(d[2]) > 1e-12:
                assert (d[2] < 0) == bool(k & 4)
            # the ray through a centre falls in that texel
            assert oracle.oct_bin(d, r)[0] == t
    assert np.all(seen == 1)
    if r == 6:
        assert [len(oracle.octant_texels(6, k)) for k in range(8)] == [6, 6, 6, 6, 3, 3, 3, 3]
    if r == 14:
        assert [len(oracle.octant_texels(14, k)) for k in range(8)] == [28] * 4 + [21] * 4


def test_dynamic_fd_closed_form_and_proxy_max():
    """One visibility trigger T at probe j, octant 3 and one radiance trigger
    R at probe m, octant 6: f_d(i, k) = Qv(i,k) (T [k=3, i within the 5x5x5
    box of j] + mu R [k=6, i within the box of m]); F is the max over each
    3x3x3 block of probes (last blocks partial)."""
    dims = (7, 4, 5)
    g = oracle.make_grid(np.zeros(3, np.float32), np.ones(3, np.float32), np.asarray(dims, np.int32))
    P = 7 * 4 * 5
    rng = np.random.default_rng(4)
    qv = rng.integers(0, 1024, P * 8).astype(np.uint16)
    tv = np.zeros(P * 8, np.int32)
    tr = np.zeros(P * 8, np.int32)
    j, m, T, R, mu = 2 + 7 * (1 + 4 * 2), 6 + 7 * (3 + 4 * 0), 700, 300, 2
    tv[8 * j + 3] = T
    tr[8 * m + 6] = R
    fd = oracle.dynamic_fd(g, mu, qv, tv, tr)

    def coords(i):
        return np.array([i % 7, (i // 7) % 4, i // 28])

    want = np.zeros(P * 8, np.int64)
    for i in range(P):
        if np.max(np.abs(coords(i) - coords(j))) <= 2:
            want[8 * i + 3] += int(qv[8 * i + 3]) * T
        if np.max(np.abs(coords(i) - coords(m))) <= 2:
            want[8 * i + 6] += int(qv[8 * i + 6]) * mu * R
    assert np.array_equal(fd, want)
    F = oracle.proxy_max(g, fd)
    pd = oracle.proxy_dims(g)
    assert pd == (3, 2, 2)
    grid = fd.reshape(5, 4, 7, 8)  # [z][y][x][octant]
    for Z in range(pd[2]):
        for Y in range(pd[1]):
            for X in range(pd[0]):
                q = X + pd[0] * (Y + pd[1] * Z)
                blk = grid[3 * Z:3 * Z + 3, 3 * Y:3 * Y + 3, 3 * X:3 * X + 3].reshape(-1, 8)
                assert np.array_equal(F[8 * q:8 * q + 8], blk.max(axis=0))


def test_dynamic_chain_targets_and_marks():
    """The dynamic chain's states settle with density proportional to F over
    (proxy region, octant), and only cells with F > 0 are marked."""
    dims = (6, 3, 3)
    g = oracle.make_grid(np.zeros(3, np.float32), np.ones(3, np.float32), np.asarray(dims, np.int32))
    pd = oracle.proxy_dims(g)
    assert pd == (2, 1, 1)
    F = np.zeros(2 * 8, np.int64)
    F[0 * 8 + 1] = 400
    F[0 * 8 + 6] = 100
    F[1 * 8 + 1] = 200
    F[1 * 8 + 4] = 300
    cp = oracle.ChainParams(512, 40, 0, 1.5, 6 * oracle.SIGMA_DIR)
    state = np.zeros((512, 5))
    occ = np.zeros(16)
    marks_seen = np.zeros(16, np.uint8)
    for frame in range(60):
        out = oracle.dyn_chain_frame(g, cp, 7, frame, F, state, init=(frame == 0))
        marks_seen |= out["mark"]
        if frame < 4:
            continue
        px = np.where(state[:, 0] < 2.5, 0, 1)  # nearest probe x < 3 -> proxy 0
        d = np.array([oracle.oct_decode(uv) for uv in state[:, 3:]])
        k = (d[:, 0] < 0).astype(int) | (d[:, 1] < 0).astype(int) << 1 | (d[:, 2] < 0).astype(int) << 2
        np.add.at(occ, 8 * px + k, 1)
    assert np.all(marks_seen[F == 0] == 0) and np.all(marks_seen[F > 0] == 1)
    # proxy regions: x in [0, 2.5] and [2.5, 5] have equal volume; octants equal area
    want = F / F.sum()
    got = occ / occ.sum()
    nz = F > 0
    # chains that started where F = 0 walk freely until they reach F > 0 and
    # never return: a vanishing share of the late states
    assert got[~nz].sum() < 2e-3
    assert np.max(np.abs(got[nz] - want[nz]) / want[nz]) < 0.08, (got, want)


def test_dynamic_rays_through_texel_centres():
    """Cornell room, fresh volume, hysteresis 0 (every update replaces the
    texel): marking one octant of one proxy updates, in each of its probes,
    exactly that octant's irradiance and depth texels once, and each depth
    texel holds tau of the ray through its centre (brute-force distance)."""
    sc = scenes.cornell()
    ora = oracle.OracleVolume(sc, seed=3, hysteresis=0.0)
    g = ora.grid
    pd = oracle.proxy_dims(g)
    assert pd == (2, 2, 2)
    mark = np.zeros(8 * 8, np.uint8)
    q, k = 5, 6  # proxy (1, 0, 1), octant (x>0, y<0, z<0)
    mark[8 * q + k] = 1
    nd = oracle.dyn_ray_counts(g, mark, 8, 16)
    base = np.ascontiguousarray(np.concatenate([[0], np.cumsum(nd)])[:-1], np.int64)
    cnt = oracle.Counts()
    oracle.lib().orc_dyn_probes_frame(
        ora.scene.ptr, oracle.C.byref(g), ora.P, oracle._p(ora.probes), oracle._p(mark), oracle._p(base),
        oracle.C.byref(ora.tol), 8, 16, 0.0, ora.tau_max, 0, None, None, oracle._p(ora.irr),
        oracle._p(ora.irr_n), oracle._p(ora.dep), oracle._p(ora.dep_n), oracle.C.byref(cnt))
    li, ld = oracle.octant_texels(6, k), oracle.octant_texels(14, k)
    s = float(np.sqrt(np.sum(np.asarray(sc.grid_spacing, np.float64) ** 2)))
    members = [i for i in range(64) if oracle.lib().orc_proxy_of_probe(oracle.C.byref(g), i) == q]
    # 4 probes per axis: blocks of 3 and 1, so proxy (1, 0, 1) holds x = 3, y = 0..2, z = 3
    assert members == [3 + 4 * (y + 4 * 3) for y in range(3)]
    assert np.all(nd[members] == len(li) + len(ld))
    assert nd.sum() == 3 * (len(li) + len(ld)) and cnt.rays == nd.sum()
    for i in range(64):
        wi = np.zeros(36, np.uint8)
        wd = np.zeros(196, np.uint8)
        if i in members:
            wi[li] = 1
            wd[ld] = 1
        assert np.array_equal(ora.irr_n[i], wi) and np.array_equal(ora.dep_n[i], wd)
    o = np.asarray(sc.grid_origin, np.float64) + 0.25 * np.array([3, 1, 3])  # probe (3,1,3) of proxy 5
    i = 3 + 4 * (1 + 4 * 3)
    for t in ld:
        h = ora.scene.closest_hit(o, oracle.texel_centre_dir(14, int(t)), brute=True)
        tau = min(h.t / s, ora.tau_max) if h.tri >= 0 else ora.tau_max
        assert abs(ora.dep[i, 2 * t] - tau) <= 1e-9 * max(tau, 1.0)


def test_quantized_static_samples_trace_texel_centres():
    """With quant set, a static sample's rays go through the centres of the
    irradiance texel of w and of the depth texel of -w: on a fresh volume with
    hysteresis 0 each touched depth texel holds tau of its centre ray."""
    sc = scenes.cornell()
    ora = oracle.OracleVolume(sc, seed=5, hysteresis=0.0)
    rng = np.random.default_rng(8)
    n = np.zeros(64, np.int32)
    n[21] = 40
    base = np.zeros(64, np.int64)
    base[22:] = 40
    uv = np.ascontiguousarray(rng.uniform(-1, 1, size=(40, 2)))
    quant = np.ones(64, np.uint8)
    cnt = oracle.Counts()
    oracle.lib().orc_chain_probes_frame(
        ora.scene.ptr, oracle.C.byref(ora.grid), 64, oracle._p(ora.probes), oracle._p(n), oracle._p(base),
        oracle._p(uv), oracle._p(quant), oracle.C.byref(ora.tol), 8, 16, 0.0, ora.tau_max, 0, None, None,
        None, None, oracle._p(ora.irr), oracle._p(ora.irr_n), oracle._p(ora.dep), oracle._p(ora.dep_n),
        oracle.C.byref(cnt))
    s = float(np.sqrt(np.sum(np.asarray(sc.grid_spacing, np.float64) ** 2)))
    o = np.asarray(sc.grid_origin, np.float64) + 0.25 * np.array([1, 1, 1])  # probe 21 = (1, 1, 1)
    touched = np.nonzero(ora.dep_n[21])[0]
    assert len(touched) > 10 and ora.dep_n[21].sum() == 40
    for t in touched:
        h = ora.scene.closest_hit(o, oracle.texel_centre_dir(14, int(t)), brute=True)
        tau = min(h.t / s, ora.tau_max) if h.tri >= 0 else ora.tau_max
        assert abs(ora.dep[21, 2 * t] - tau) <= 1e-9 * max(tau, 1.0)


def test_chain_update_with_dynamic_chains_runs_end_to_end():
    """A chain frame with dynamic chains after a light change: detection
    marks proxies, every probe of a marked proxy gets its octants' texel
    rays, and the ray count adds up."""
    sc = scenes.cornell()
    sc.light_a = np.array([[0.5, 0.95, 0.5]], np.float32)
    sc.light_b = np.array([[0.2, 0.5, 0.3]], np.float32)
    sc.frames = 6
    ora = oracle.OracleVolume(sc, seed=9)
    cp = oracle.ChainParams(64, 12, 3, 0.5, oracle.SIGMA_DIR)
    dp = oracle.ChainParams(32, 12, 3, 1.5, 6 * oracle.SIGMA_DIR)
    st, dst = np.zeros((64, 5)), np.zeros((32, 5))
    for f in range(4):
        out = ora.chain_update(f, cp, st, init=(f == 0), dyn=dp, dyn_state=dst, dyn_init=(f == 0))
        R = int(out["dyn_rays"].sum())
        assert out["counts"]["rays"] == 2 * 64 * 8 + R + 8 * ora.P  # samples, dynamic rays, pilots
        assert np.all(out["mark"][out["F"] == 0] == 0)
        if f == 3:
            assert out["F"].max() > 0 and out["mark"].sum() > 0 and R > 0
            assert np.array_equal(out["score"] > 0, out["fd"].reshape(-1, 8).sum(axis=1) > 0)


# ---- DDGI cosine-weighted gather (the blend of Sec. 3.1, Majercik et al. 2019)

def _sky_over_black_plane(height=0.5):
    s = 1e4
    pos = np.array([[-s, -s, 0.0], [s, -s, 0.0], [s, s, 0.0], [-s, s, 0.0]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return scenes.Scene(name="plane", positions=pos, indices=idx, albedo=np.zeros((2, 3), np.float32),
                        light_a=np.zeros((0, 3), np.float32), light_b=np.zeros((0, 3), np.float32),
                        light_intensity=np.zeros((0, 3), np.float32), sky=np.array([0.8, 0.5, 0.2], np.float32),
                        grid_origin=np.array([0.0, 0.0, height], np.float32),
                        grid_spacing=np.array([1.0, 1.0, 1.0], np.float32),
                        grid_dims=np.array([1, 1, 1], np.int32), frames=2)


def test_gather_sky_fraction_closed_form():
    """A probe over a black plane under a uniform sky: the cosine-weighted
    mean radiance of a texel with centre direction c is sky * (1 + c_z) / 2
    (the sky's view factor for a surface tilted from +z), reached by 8192
    spherical-Fibonacci rays to within 2e-3 of the sky; depth texels whose
    lobe sees only sky hold (tau_max, tau_max^2)."""
    sc = _sky_over_black_plane()
    ora = oracle.OracleVolume(sc, seed=3, gather=True, hysteresis=0.97)
    ora.update(0, adaptive=False, n_uniform=8192)
    sky = np.asarray(sc.sky, np.float64)
    for k in range(36):
        c = oracle.texel_centre_dir(6, k)
        want = sky * (1.0 + c[2]) / 2.0
        assert np.all(np.abs(ora.irr[0, 3 * k:3 * k + 3] - want) <= 2e-3 * sky.max()), (k, c)
    assert np.all(ora.irr_n[0] == 1)
    for k in range(196):
        c = oracle.texel_centre_dir(14, k)
        if c[2] > 0.9:  # the cos^50 lobe (about 10 degrees wide) sees the horizon below 1e-18
            assert abs(ora.dep[0, 2 * k] - ora.tau_max) < 1e-9 * ora.tau_max
            assert abs(ora.dep[0, 2 * k + 1] - ora.tau_max ** 2) < 1e-9 * ora.tau_max ** 2


def test_gather_step_rule_counts_frames():
    """Second frame under another sky: every texel moves halfway
    (a = max(1/(N+1), 1-h) = 1/2 with N = 1 frame), counts reach 2."""
    sc = _sky_over_black_plane()
    ora = oracle.OracleVolume(sc, seed=3, gather=True, hysteresis=0.97)
    ora.update(0, adaptive=False, n_uniform=512)
    first = ora.irr.copy()
    sc.sky = np.array([0.1, 0.3, 0.9], np.float32)
    ora.update(1, adaptive=False, n_uniform=512)
    # the second frame's own mean under the new sky, from a fresh volume
    fresh = oracle.OracleVolume(sc, seed=3, gather=True, hysteresis=0.97)
    fresh.update(1, adaptive=False, n_uniform=512)
    assert np.allclose(ora.irr, first + 0.5 * (fresh.irr - first), rtol=0, atol=1e-12)
    assert np.all(ora.irr_n == 2)


# ---- irradiance query (the 8-probe lookup of Sec. 3.1, DDGI's weights)

def _query_grid(dims, spacing=1.0):
    return oracle.make_grid(np.zeros(3, np.float32), np.full(3, spacing, np.float32), np.asarray(dims, np.int32))


def _tiles(P, value_irr, value_dep):
    irr = np.broadcast_to(np.asarray(value_irr, np.float64), (P, 8, 8, 3)).copy()
    dep = np.broadcast_to(np.asarray(value_dep, np.float64), (P, 16, 16, 2)).copy()
    return irr, dep


def test_query_constant_field():
    """Every probe holding the same irradiance c gives c anywhere, for any
    normal and any visibility (the weights are normalised)."""
    g = _query_grid((3, 2, 4))
    rng = np.random.default_rng(1)
    irr, dep = _tiles(24, [0.3, 0.5, 0.7], [0.2, 0.05])
    pts = rng.uniform([-0.5, -0.5, -0.5], [2.5, 1.5, 3.5], size=(50, 3))
    nrm = rng.normal(size=(50, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    out = oracle.query_irradiance(g, irr, dep, pts, nrm)
    assert np.allclose(out, [0.3, 0.5, 0.7], rtol=0, atol=1e-12)


def test_query_linear_between_two_visible_probes():
    """Two probes along x, normal along y (both probes at the same backface
    angle), no occluder: the query is the linear interpolation of the two
    probes' irradiance in direction n."""
    g = _query_grid((2, 1, 1))
    irr, dep = _tiles(2, [0.0, 0.0, 0.0], [50.0, 2500.0])
    irr[0] = [0.2, 0.4, 0.6]
    irr[1] = [1.0, 0.1, 0.3]
    for a in (0.0, 0.25, 0.6, 1.0):
        out = oracle.query_irradiance(g, irr, dep, [[a, 0.0, 0.0]], [[0.0, 1.0, 0.0]])[0]
        assert np.allclose(out, (1 - a) * irr[0, 0, 0] + a * irr[1, 0, 0], rtol=0, atol=1e-12), a


def test_query_chebyshev_hides_an_occluded_probe():
    """Probe 0 saw a wall at distance 0.1 s in every direction (variance 0):
    a point halfway to probe 1 is occluded from probe 0, so the query returns
    probe 1's irradiance up to the 1e-6 weight floor."""
    g = _query_grid((2, 1, 1))
    irr, dep = _tiles(2, [0.0, 0.0, 0.0], [50.0, 2500.0])
    irr[0] = [5.0, 5.0, 5.0]
    irr[1] = [0.3, 0.2, 0.1]
    dep[0] = [0.1, 0.01]
    out = oracle.query_irradiance(g, irr, dep, [[0.5, 0.0, 0.0]], [[0.0, 0.0, 1.0]])[0]
    assert np.allclose(out, [0.3, 0.2, 0.1], rtol=0, atol=5e-5 * 5.0)
    # and without the wall the first probe counts in full again
    dep[0] = [50.0, 2500.0]
    out = oracle.query_irradiance(g, irr, dep, [[0.5, 0.0, 0.0]], [[0.0, 0.0, 1.0]])[0]
    assert np.allclose(out, 0.5 * (irr[0, 0, 0] + irr[1, 0, 0]), rtol=0, atol=1e-12)


def test_query_at_a_probe_reads_its_texel():
    """Just off a probe along n, with n through the centre of interior texel
    k, the query returns that probe's texel k (bilinear at a texel centre)."""
    g = _query_grid((3, 3, 3))
    rng = np.random.default_rng(6)
    ri = 6
    interior = rng.uniform(0.1, 1.0, size=(27, ri * ri * 3))
    irr = np.stack([oracle.fold_tile(t, ri, 3).reshape(8, 8, 3) for t in interior])
    dep = np.broadcast_to(np.asarray([50.0, 2500.0]), (27, 16, 16, 2)).copy()
    p = 1 + 3 * (1 + 3 * 1)  # probe (1, 1, 1) at (1, 1, 1)
    for k in (0, 7, 14, 21, 35):
        n = oracle.texel_centre_dir(ri, k)
        x = np.array([1.0, 1.0, 1.0]) + 1e-9 * n
        out = oracle.query_irradiance(g, irr, dep, [x], [n])[0]
        assert np.allclose(out, interior[p, 3 * k:3 * k + 3], rtol=0, atol=1e-7), k
