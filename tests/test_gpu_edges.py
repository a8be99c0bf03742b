"""Edge cases of the probe update on the GPU, each against the oracle in
lockstep and, where one exists, against a closed form (needs an MI355X).

Covers the empty scene under a uniform sky (every sampled texel is the sky
exactly, every depth texel tau_max), a budget at or above P * n_max, n_min =
n_max, scenes without lights, a single-probe grid and probe counts that are
not multiples of the 64-lane wave.
"""
import numpy as np
import pytest

import oracle
import scenes
from tests.parity import run_lockstep
from tests.test_gpu_parity import _assert_parity

pytestmark = pytest.mark.gpu

SKY = np.array([0.7, 1.3, 2.0], np.float32)


def _empty_scene(dims):
    sc = scenes.cornell()
    return scenes.Scene(
        name="empty", positions=np.zeros((0, 3), np.float32), indices=np.zeros((0, 3), np.int32),
        albedo=np.zeros((0, 3), np.float32), light_a=np.zeros((0, 3), np.float32),
        light_b=np.zeros((0, 3), np.float32), light_intensity=np.zeros((0, 3), np.float32),
        sky=SKY.copy(), grid_origin=sc.grid_origin, grid_spacing=sc.grid_spacing,
        grid_dims=np.array(dims, np.int32), frames=4)


def _gpu_run(scene, frames, **kw):
    """Frames on the GPU alone; returns the last readback."""
    import paper_2301_05125_amd as adgi
    P = scene.num_probes
    vol = adgi.volume_for_scene(scene, max_rays=max(kw.get("budget", 0), P * kw.get("n_uniform", 1)),
                                seed=0x5EED, debug=True)
    bins = np.zeros((P, 36), np.int64)
    for f in range(frames):
        vol.update_probes(f, sync=True, **kw)
        rb = vol.read_probes(texels=True, debug=True)
        off = rb["ray_offsets"]
        for i in range(P):
            bins[i] += np.bincount(rb["irr_bin"][off[i]:off[i + 1]], minlength=36)
    vol.destroy_volume()
    return rb, bins


def test_pin1_empty_scene_uniform_sky_on_gpu():
    """No triangles, uniform sky, 3x5x7 = 105 probes (not a multiple of 64),
    97 rays per probe: every sampled irradiance texel equals the sky exactly
    (the first sample has step 1, later samples change nothing), every
    sampled depth texel holds tau_max and tau_max^2 (FP32 product), counts
    equal the samples per texel, unsampled texels stay 0; and the oracle
    agrees in lockstep."""
    sc = _empty_scene((3, 5, 7))
    rb, bins = _gpu_run(sc, 3, adaptive=False, n_uniform=97)
    ri = rb["irradiance"][:, 1:-1, 1:-1].reshape(105, 36, 3)
    cnt = rb["irr_count"].reshape(105, 36)
    assert np.array_equal(cnt, np.minimum(bins, 255))
    hit = cnt > 0
    assert np.all(ri[hit] == SKY[None, :]) and np.all(ri[~hit] == 0)
    tau = np.float32(oracle.TAU_MAX)
    dep = rb["depth"][:, 1:-1, 1:-1].reshape(105, 196, 2)
    dh = rb["depth_count"].reshape(105, 196) > 0
    assert np.all(dep[dh][:, 0] == tau) and np.all(dep[dh][:, 1] == np.float32(tau * tau))
    res = run_lockstep(sc, frames=3, adaptive=False, n_uniform=97)
    _assert_parity(res)


def test_empty_scene_adaptive_is_uniform_split():
    """Empty scene, adaptive: pilots all miss, the sky never changes, every
    score is 0, so the budget splits evenly with the remainder one ray each
    to the lowest-index probes: n_i = n_min + floor(B'/P) + [i < B' mod P]."""
    sc = _empty_scene((3, 5, 7))
    P, n_min, n_max = 105, 8, 64
    B = P * 20 + 17
    rb, _ = _gpu_run(sc, 4, adaptive=True, budget=B, n_min=n_min, n_max=n_max)
    Bp = B - P * n_min
    expect = n_min + Bp // P + (np.arange(P) < Bp % P)
    assert np.array_equal(rb["rays_per_probe"], expect)
    assert np.all(rb["score"] == 0)
    assert np.all(rb["q10_vis"] == 0)
    # sky luminance (Rec. 709) 1.2226... -> floor(1024 * 1.2226 / 5) = 250
    lum = 0.2126 * 0.7 + 0.7152 * 1.3 + 0.0722 * 2.0
    assert np.all(rb["q10_rad"] == int(np.floor(1024 * lum / 5)))
    res = run_lockstep(sc, frames=4, adaptive=True, budget=B, n_min=n_min, n_max=n_max)
    _assert_parity(res)


def _moving_light_cornell(dims=None):
    sc = scenes.cornell()
    sc.light_a = np.array([[0.5, 0.95, 0.5]], np.float32)
    sc.light_b = np.array([[0.2, 0.5, 0.3]], np.float32)
    sc.frames = 6
    if dims is not None:
        sc.grid_dims = np.array(dims, np.int32)
        sc.grid_spacing = (1.0 / sc.grid_dims).astype(np.float32)
        sc.grid_origin = (0.5 * sc.grid_spacing).astype(np.float32)
    return sc


@pytest.mark.parametrize("extra", [0, 1000])
def test_saturated_budget(extra):
    """B >= P * n_max: lambda* is the top of its range, no probe exceeds
    n_max, the total never exceeds B, and the allocation equals the
    oracle's exactly (the split is integer arithmetic on the scores)."""
    sc = _moving_light_cornell()
    P, n_min, n_max = sc.num_probes, 8, 96
    B = P * n_max + extra
    res = run_lockstep(sc, frames=6, adaptive=True, budget=B, n_min=n_min, n_max=n_max)
    _assert_parity(res)
    n = res["stats_last"]
    assert n["budget_used"] <= B and n["n_max_seen"] <= n_max and n["n_min_seen"] >= n_min


def test_n_min_equals_n_max():
    """n_min = n_max: every probe traces exactly that many rays whatever its
    score."""
    sc = _moving_light_cornell()
    P, n = sc.num_probes, 40
    res = run_lockstep(sc, frames=4, adaptive=True, budget=P * n, n_min=n, n_max=n)
    _assert_parity(res)
    st = res["stats_last"]
    assert st["n_min_seen"] == n and st["n_max_seen"] == n and st["budget_used"] == P * n


def test_no_lights_sky_only():
    """A small box field with no lights and a coloured sky: hits are black,
    misses carry the sky; adaptive frames on 5 x 3 x 7 = 105 probes."""
    sc = scenes.box_field(seed=scenes.SEED_BASE + 310, lattice=16, dims=(5, 3, 7), n_lights=1, frames=6)
    sc.light_a = np.zeros((0, 3), np.float32)
    sc.light_b = np.zeros((0, 3), np.float32)
    sc.light_intensity = np.zeros((0, 3), np.float32)
    sc.sky = np.array([0.3, 0.5, 0.9], np.float32)
    P = sc.num_probes
    res = run_lockstep(sc, frames=4, adaptive=True, budget=P * 48, n_min=8, n_max=256)
    _assert_parity(res)
    assert res["oracle_counts"]["rays"] > 0


def test_single_probe_grid():
    """A 1 x 1 x 1 grid in the Cornell room (the 5x5x5 sum holds only the
    probe itself): uniform frames, then adaptive frames whose whole budget
    goes to the one probe (n = min(n_max, B))."""
    sc = _moving_light_cornell(dims=(1, 1, 1))
    res = run_lockstep(sc, frames=3, adaptive=False, n_uniform=200)
    _assert_parity(res)
    res = run_lockstep(sc, frames=6, adaptive=True, budget=300, n_min=8, n_max=512)
    _assert_parity(res)
    assert res["stats_last"]["budget_used"] == 300
