"""adgi_update_probes_static against adgi_update_probes (needs an MI355X).

The static variant runs the same kernels with the frame scratch carved from
the library's fixed per-GPU array, so every output of a frame (texels,
counts, allocation, scores, detection codes, ray records, per-ray and
per-pilot decisions, frame counters) must equal the allocating entry point's
bit for bit. Two calls in a row: frames of a 2048-probe budgeted volume
(B = 2^19, pilot reuse), then frames of a 64-probe uniform volume, whose
smaller frame leaves most of the array holding the first volume's leftovers.
"""
import ctypes as C

import numpy as np
import pytest

import scenes
from tests.parity import gpu_scene_update

pytestmark = pytest.mark.gpu


def _adgi():
    import paper_2301_05125_amd as adgi
    return adgi


def _same(a, b, what):
    assert a.keys() == b.keys(), what
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, np.ndarray):
            assert x.dtype == y.dtype and x.shape == y.shape, (what, k)
            assert x.tobytes() == y.tobytes(), f"{what}: {k} differs"
        else:
            assert x == y, (what, k, x, y)


def _stats(st):
    return {k: v for k, v in st.items() if not k.startswith("ms")}


def _pair(scene, max_rays, static_flag):
    adgi = _adgi()
    a = adgi.volume_for_scene(scene, max_rays=max_rays, seed=0x5EED, debug=True)
    b = adgi.volume_for_scene(scene, max_rays=max_rays, seed=0x5EED, debug=True, static_scratch=static_flag)
    return a, b


def _run_and_compare(scene, a, b, frames, **kw):
    for f in range(frames):
        if f > 0:
            gpu_scene_update(a, scene, f)
            gpu_scene_update(b, scene, f)
        sa = a.update_probes(f, sync=True, **kw)
        sb = b.update_probes_static(f, sync=True, **kw)
        assert _stats(sa) == _stats(sb), f
        _same(a.read_probes(texels=True, debug=True), b.read_probes(texels=True, debug=True), f"frame {f}")


def test_static_scratch_matches_update_probes_two_calls():
    adgi = _adgi()
    big = scenes.box_field(seed=scenes.SEED_BASE + 311, lattice=24, dims=(16, 8, 16), n_lights=2, frames=6)
    B = 1 << 19
    a, b = _pair(big, B, static_flag=True)
    try:
        assert adgi.lib().adgi_device_bytes(b.h) < adgi.lib().adgi_device_bytes(a.h)
        _run_and_compare(big, a, b, 4, adaptive=True, budget=B, n_min=32, n_max=1024, pilot_reuse=True)
    finally:
        a.destroy_volume()
        b.destroy_volume()
    small = scenes.cornell()
    # an ordinary volume may use the static entry point too
    c, d = _pair(small, small.num_probes * 64, static_flag=False)
    try:
        _run_and_compare(small, c, d, 3, adaptive=False, n_uniform=64)
        # and go back and forth between the two entry points on one volume
        gpu_scene_update(c, small, 3)
        gpu_scene_update(d, small, 3)
        sa = c.update_probes(3, adaptive=True, budget=small.num_probes * 40, n_min=8, n_max=256, sync=True)
        sb = d.update_probes(3, adaptive=True, budget=small.num_probes * 40, n_min=8, n_max=256, sync=True)
        assert _stats(sa) == _stats(sb)
        _same(c.read_probes(texels=True, debug=True), d.read_probes(texels=True, debug=True), "frame 3")
    finally:
        c.destroy_volume()
        d.destroy_volume()


def test_static_scratch_rejections():
    adgi = _adgi()
    sc = scenes.cornell()
    P = sc.num_probes
    # a static-scratch volume has no frame scratch of its own
    v = adgi.volume_for_scene(sc, max_rays=P * 64, static_scratch=True)
    try:
        with pytest.raises(adgi.AdgiError) as e:
            v.update_probes(0, adaptive=False, n_uniform=64)
        assert e.value.status == adgi.ADGI_ERR_INVALID_ARG
        v.update_probes_static(0, adaptive=False, n_uniform=64)
    finally:
        v.destroy_volume()
    # frames whose scratch exceeds the array: rejected before anything runs
    big_rays = adgi.ADGI_STATIC_SCRATCH_BYTES // 56 + 4096
    v = adgi.volume_for_scene(sc, max_rays=big_rays, static_scratch=True)
    try:
        with pytest.raises(adgi.AdgiError) as e:
            v.update_probes_static(0, adaptive=True, budget=big_rays, n_min=8, n_max=65535)
        assert e.value.status == adgi.ADGI_ERR_BUDGET
        st = v.update_probes_static(0, adaptive=True, budget=P * 64, n_min=8, n_max=256)
        assert st["budget_used"] <= P * 64
    finally:
        v.destroy_volume()
    # chain frames go through adgi_update_probes only
    v = adgi.volume_for_scene(sc, max_rays=P * 64, max_chains=64)
    try:
        p = adgi.Volume._chain_params(0, 64, 8, 2, 0.5, adgi.CHAIN_SIGMA_DIR, True, 5.0, True)
        assert adgi.lib().adgi_update_probes_static(v.h, C.byref(p), None) == adgi.ADGI_ERR_INVALID_ARG
    finally:
        v.destroy_volume()
    with pytest.raises(adgi.AdgiError) as e:
        adgi.volume_for_scene(sc, max_rays=P * 64, max_chains=64, static_scratch=True)
    assert e.value.status == adgi.ADGI_ERR_INVALID_ARG
