"""Runtime behaviour of the library on the GPU: determinism across runs,
launch shapes and graph/eager execution, snapshots, and error paths."""
import numpy as np
import pytest

import paper_2301_05125_amd as adgi
import scenes

pytestmark = pytest.mark.gpu


def _run(sc, frames, adaptive, tuning=None, budget=0, n_min=8, n_max=256, n_uniform=64,
         storage=adgi.ADGI_FP32, seed=3, vol=None, start=0):
    own = vol is None
    if own:
        vol = adgi.volume_for_scene(sc, storage=storage, max_rays=max(budget, sc.num_probes * n_uniform),
                                    seed=seed)
    if tuning:
        vol.set_tuning(**tuning)
    for f in range(start, start + frames):
        vol.update_scene(sc.positions_at(f), light_pos=sc.light_positions(f),
                         light_intensity=sc.light_intensity, sky=sc.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, sc.anim_vertices))
        vol.update_probes(f, adaptive=adaptive, budget=budget, n_min=n_min, n_max=n_max,
                          n_uniform=n_uniform, sync=True)
    rb = vol.read_probes()
    if own:
        vol.destroy_volume()
    return rb


def _small_field():
    return scenes.box_field(lattice=48, dims=(16, 4, 16), frames=8)


def _same(a, b):
    for k in ("irradiance", "depth", "irr_count", "depth_count", "rays_per_probe", "score",
              "q10_vis", "q10_rad", "irr_words", "depth_words"):
        if k in a or k in b:
            if not np.array_equal(a[k], b[k], equal_nan=a[k].dtype.kind == "f"):
                bad = np.argwhere(a[k] != b[k])
                raise AssertionError(f"{k}: {len(bad)} elements differ, first {bad[:4].tolist()}, "
                                     f"max |diff| {np.max(np.abs(a[k].astype(np.float64) - b[k])):.3g}")


def test_bitwise_determinism_across_runs():
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    _same(_run(sc, 6, **kw), _run(sc, 6, **kw))


def test_later_volumes_reuse_released_streams():
    """The streams of a destroyed volume go to the next one created (its
    events are new): volumes made one after another, each running more
    graph frames than its parameter ring has slots, agree bit for bit."""
    sc = scenes.box_field(lattice=48, dims=(16, 4, 16), frames=12)
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    first = _run(sc, 10, **kw)
    for _ in range(3):
        _same(first, _run(sc, 10, **kw))


def test_large_ray_buffers_take_the_multi_block_pair_scan():
    """A volume whose ray buffers hold more than 2^14 batches of 64 rays lays
    out the shadow pairs with the three-launch scan; the frames must match a
    volume sized to the budget (one-workgroup scan) bit for bit."""
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    big = adgi.volume_for_scene(sc, max_rays=(1 << 20) + 64 * 1024, seed=3)
    try:
        a = _run(sc, 4, vol=big, **kw)
    finally:
        big.destroy_volume()
    _same(a, _run(sc, 4, **kw))


@pytest.mark.parametrize("tuning", [{"use_graph": 0}, {"bvh_width": 4, "trace_block": 128}])
def test_packed_storage_launch_invariance(tuning):
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256, storage=adgi.ADGI_PACKED)
    a, b = _run(sc, 4, **kw), _run(sc, 4, tuning=tuning, **kw)
    _same(a, b)


@pytest.mark.parametrize("tuning", [
    {"use_graph": 0},
    {"persistent": 0},
    {"trace_block": 64, "trace_waves_per_cu": 8},
    {"trace_block": 256, "trace_waves_per_cu": 16},
    {"blend_chunk": 64},
    {"blend_chunk": 512},
    {"bvh_width": 2},
    {"bvh_width": 2, "persistent": 0},
    {"bvh_width": 2, "trace_block": 128},
    {"ray_order": 0},
    {"ray_order": 0, "bvh_width": 2, "persistent": 0},
])
def test_launch_shape_does_not_change_results(tuning):
    """Frames, pilot codes included, are bitwise the same for every launch
    shape. The 1,024 probes' 8,192 pilots go 1, 4 and 2 to a wave at 32, 8
    and 16 waves per CU (a pilot pass halves its batches until it fills the
    launch), so the pilot batch size varies here too."""
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    _same(_run(sc, 4, **kw), _run(sc, 4, tuning=tuning, **kw))


def test_refit_of_a_vertex_range_matches_a_full_refit():
    """A REFIT that names the moved vertices rebuilds only the triangles that
    touch them; frames after it match those after refits of every vertex, bit
    for bit (ray records and hit triangles included), also when the range
    changes from frame to frame and right after a REBUILD."""
    sc = _small_field()
    P = sc.num_probes

    def refit(vol, f, rng):
        vol.update_scene(sc.positions_at(f), light_pos=sc.light_positions(f),
                         light_intensity=sc.light_intensity, sky=sc.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=rng)

    def run(ranged):
        vol = adgi.volume_for_scene(sc, max_rays=P * 64, seed=3, debug=True)
        out = []
        for f in range(6):
            if f == 3:  # a REBUILD mid-way: the next refit must redo every triangle
                vol.update_scene(sc.positions_at(f), sc.indices, albedo=sc.albedo,
                                 light_pos=sc.light_positions(f), light_intensity=sc.light_intensity,
                                 sky=sc.sky, mode=adgi.ADGI_SCENE_REBUILD)
            if not ranged:
                refit(vol, f, (0, sc.positions.shape[0]))
            elif f == 2:  # half the moving vertices, then the rest
                refit(vol, f, (0, sc.anim_vertices // 2))
                refit(vol, f, (sc.anim_vertices // 2, sc.anim_vertices))
            else:
                refit(vol, f, (0, sc.anim_vertices))
            vol.update_probes(f, adaptive=False, n_uniform=64, sync=True)
            rb = vol.read_probes(debug=True)
            out.append([rb[k].copy() for k in ("irradiance", "depth", "hit_tri", "ray_record")])
        vol.destroy_volume()
        return out

    assert sc.anim_vertices > 0
    a, b = run(True), run(False)
    for fa, fb in zip(a, b):
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)


def test_autotune_keeps_state_and_results():
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    ref = _run(sc, 4, **kw)
    vol = adgi.volume_for_scene(sc, max_rays=sc.num_probes * 40, seed=3)
    _run(sc, 2, vol=vol, **kw)
    before = vol.read_probes()
    chosen = vol.autotune(2, **kw)
    assert chosen["trace_block"] in (64, 128, 256)
    after = vol.read_probes()
    _same(before, after)
    out = _run(sc, 2, vol=vol, start=2, **kw)
    vol.destroy_volume()
    _same(ref, out)


@pytest.mark.parametrize("width", [2, 4])
def test_trace_work_counts(width):
    """The work-counting run traces the frame's own probe rays and leaves
    the state alone: on a uniform frame (no pilots, whose shadow rays the
    frame's statistics would include) its ray counts equal those of the
    frame that follows; a BVH2 visit tests two child boxes, a BVH4 visit
    between one and four (empty slots not counted), and the shading
    kernel's share is part of the totals."""
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256)
    vol = adgi.volume_for_scene(sc, max_rays=sc.num_probes * 40, seed=3)
    vol.set_tuning(bvh_width=width)
    _run(sc, 2, vol=vol, **kw)
    vol.update_scene(sc.positions_at(2), light_pos=sc.light_positions(2), light_intensity=sc.light_intensity,
                     sky=sc.sky, mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, sc.anim_vertices))
    before = vol.read_probes()
    assert vol.measure_trace_work(2, **kw)["primary_rays"] == sc.num_probes * 40
    _same(before, vol.read_probes())
    ku = dict(adaptive=False, n_uniform=40)
    tw = vol.measure_trace_work(2, **ku)
    _same(before, vol.read_probes())
    st = vol.update_probes(2, sync=True, **ku)
    vol.destroy_volume()
    assert tw["primary_rays"] == st["primary_rays"] and tw["shadow_rays"] == st["shadow_rays"]
    assert tw["node_tests"] > tw["shade_node_tests"] > 0 and tw["tri_tests"] > tw["shade_tri_tests"] > 0
    assert 0 < tw["shade_box_tests"] < tw["box_tests"]
    if width == 2:
        assert tw["box_tests"] == 2 * tw["node_tests"] and tw["shade_box_tests"] == 2 * tw["shade_node_tests"]
    else:
        assert tw["node_tests"] <= tw["box_tests"] <= 4 * tw["node_tests"]


@pytest.mark.parametrize("storage", [adgi.ADGI_FP32, adgi.ADGI_PACKED])
def test_snapshot_resumes_bit_identically(storage):
    sc = _small_field()
    kw = dict(adaptive=True, budget=sc.num_probes * 40, n_min=8, n_max=256, storage=storage)
    ref = _run(sc, 6, **kw)
    v1 = adgi.volume_for_scene(sc, max_rays=sc.num_probes * 40, seed=3, storage=storage)
    _run(sc, 3, vol=v1, **kw)
    snap = v1.save_state()
    v1.destroy_volume()
    v2 = adgi.volume_for_scene(sc, max_rays=sc.num_probes * 40, seed=3, storage=storage)
    v2.restore_state(snap)
    out = _run(sc, 3, vol=v2, start=3, **kw)
    v2.destroy_volume()
    _same(ref, out)


def test_error_paths():
    sc = scenes.cornell()
    vol = adgi.Volume(sc.grid_origin, sc.grid_spacing, sc.grid_dims, max_rays_per_frame=64 * 64)
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_probes(0, adaptive=False, n_uniform=64)
    assert e.value.status == -4  # no scene
    vol.update_scene(sc.positions, sc.indices, sc.albedo, sc.light_positions(0),
                     sc.light_intensity, sc.sky)
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_probes(0, adaptive=True, budget=64 * 8 - 1, n_min=8, n_max=64)
    assert e.value.status == -3  # budget below P * n_min
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_probes(0, adaptive=False, n_uniform=65)
    assert e.value.status == -3  # over max_rays_per_frame
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_scene(sc.positions[:-1], light_pos=sc.light_positions(0),
                         light_intensity=sc.light_intensity, mode=adgi.ADGI_SCENE_REFIT)
    assert e.value.status == -5  # topology change
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_scene(sc.positions, sc.indices, sc.albedo, np.zeros((9, 3)), np.ones((9, 3)))
    assert e.value.status == -1  # too many lights
    # the volume is unchanged and still works after every rejected call
    vol.update_probes(0, adaptive=False, n_uniform=64)
    rb = vol.read_probes()
    assert rb["irr_count"].sum() > 0
    vol.destroy_volume()


def test_allocator_failure_reports_out_of_memory():
    calls = {"n": 0}

    def alloc(nbytes, ctx):
        calls["n"] += 1
        if calls["n"] > 5:
            return None
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def free(ptr, ctx):
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))

    a = adgi.Allocator(adgi.ALLOC_FN(alloc), adgi.FREE_FN(free), None)
    sc = scenes.cornell()
    with pytest.raises(adgi.AdgiError) as e:
        adgi.Volume(sc.grid_origin, sc.grid_spacing, sc.grid_dims, allocator=a)
    assert e.value.status == -2


# ---- chain frames

def _chain_run(sc, frames, tuning=None, vol=None, start=0, chains=768, steps=24, burn_in=5):
    own = vol is None
    if own:
        vol = adgi.volume_for_scene(sc, max_rays=max(2 * chains * steps, sc.num_probes * 32), seed=5,
                                    max_chains=chains)
    if tuning:
        vol.set_tuning(**tuning)
    for f in range(start, start + frames):
        vol.update_scene(sc.positions_at(f), light_pos=sc.light_positions(f),
                         light_intensity=sc.light_intensity, sky=sc.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, sc.anim_vertices))
        if f < 1:
            vol.update_probes(f, adaptive=False, n_uniform=32, sync=True)
        else:
            st = vol.update_chains(f, chains, steps, burn_in, sync=True)
            assert st["primary_rays"] == 2 * chains * (steps - burn_in - 1)
            assert st["pilot_rays"] == 8 * sc.num_probes
    rb = vol.read_probes()
    if own:
        vol.destroy_volume()
    return rb


def _same_chain(a, b):
    _same(a, b)
    for k in ("chain_state", "sample_probe", "sample_uv"):
        assert np.array_equal(a[k], b[k]), (k, int(np.count_nonzero(a[k] != b[k])))


@pytest.mark.parametrize("tuning", [
    {"use_graph": 0},
    {"persistent": 0},
    {"trace_block": 256, "trace_waves_per_cu": 16},
    {"bvh_width": 4},
    {"blend_blocks_per_cu": 4},
    {"chain_lanes": 1},
    {"chain_lanes": 4},
    {"chain_lanes": 8},
    {"chain_lanes": 32},
])
def test_chain_launch_shape_does_not_change_results(tuning):
    """Every launch shape, eager frames against the captured frame graphs
    (the default), and the one-thread-per-chain kernel against the
    prefetching groups (16 lanes for 768 chains by default), give the same
    chains and texels bit for bit."""
    sc = _small_field()
    _same_chain(_chain_run(sc, 4), _chain_run(sc, 4, tuning=tuning))


def test_chain_snapshot_resumes_bit_identically():
    sc = _small_field()
    ref = _chain_run(sc, 5)
    vol = adgi.volume_for_scene(sc, max_rays=2 * 768 * 24, seed=5, max_chains=768)
    _chain_run(sc, 3, vol=vol)
    snap = vol.save_state()
    vol.destroy_volume()
    vol2 = adgi.volume_for_scene(sc, max_rays=2 * 768 * 24, seed=5, max_chains=768)
    vol2.restore_state(snap)
    got = _chain_run(sc, 2, vol=vol2, start=3)
    vol2.destroy_volume()
    _same_chain(ref, got)


def test_chain_graph_follows_shape_changes():
    """A chain frame graph is taken per frame parity and replayed only for the
    shape it was taken at: changing the chain count, the samples per chain
    and switching dynamic chains on and off between frames gives the same
    chains and texels as eager frames, bit for bit."""
    sc = _small_field()
    seq = [(512, 20, 3, 0), (512, 20, 3, 0), (768, 20, 3, 0), (768, 24, 3, 64), (768, 24, 3, 64),
           (512, 20, 3, 0), (512, 20, 3, 0)]

    def run(use_graph):
        vol = adgi.volume_for_scene(sc, max_rays=2 * 768 * 24 + sc.num_probes * 232, seed=4, max_chains=768)
        vol.set_tuning(use_graph=use_graph)
        vol.update_probes(0, adaptive=False, n_uniform=32, sync=True)
        for f, (c, m, k, dyn) in enumerate(seq, start=1):
            vol.update_scene(sc.positions_at(f), light_pos=sc.light_positions(f),
                             light_intensity=sc.light_intensity, sky=sc.sky,
                             mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, sc.anim_vertices))
            kw = dict(dyn_chains=dyn, dyn_steps=12, dyn_burn_in=2) if dyn else {}
            vol.update_chains(f, c, m, k, sync=True, **kw)
        rb = vol.read_probes()
        vol.destroy_volume()
        return rb

    _same_chain(run(0), run(1))


def test_chain_and_budgeted_frames_interleave():
    """A budgeted frame between chain frames leaves the chains where they
    stopped; the sequence is deterministic."""
    sc = _small_field()

    def run():
        vol = adgi.volume_for_scene(sc, max_rays=1 << 16, seed=9, max_chains=512)
        vol.update_probes(0, adaptive=False, n_uniform=16, sync=True)
        vol.update_chains(1, 512, 20, 3, sync=True)
        s1 = vol.read_probes(texels=False)["chain_state"].copy()
        vol.update_probes(2, adaptive=True, budget=sc.num_probes * 16, n_min=4, n_max=64, sync=True)
        s2 = vol.read_probes(texels=False)["chain_state"].copy()
        vol.update_chains(3, 512, 20, 3, sync=True)
        rb = vol.read_probes()
        vol.destroy_volume()
        return s1, s2, rb

    a1, a2, ra = run()
    b1, b2, rb = run()
    assert np.array_equal(a1, a2)
    assert np.array_equal(a1, b1)
    _same_chain(ra, rb)


def test_chain_error_paths():
    sc = scenes.box_field(seed=scenes.SEED_BASE + 210, lattice=16, dims=(8, 2, 8), n_lights=1,
                          frames=2)
    plain = adgi.volume_for_scene(sc, max_rays=4096)
    with pytest.raises(adgi.AdgiError) as e:
        plain.update_chains(0, 16, 8, 1)
    assert e.value.status == adgi.ADGI_ERR_INVALID_ARG
    plain.destroy_volume()
    with pytest.raises(adgi.AdgiError) as e:
        adgi.volume_for_scene(sc, storage=adgi.ADGI_PACKED, max_rays=4096, max_chains=16)
    assert e.value.status == adgi.ADGI_ERR_INVALID_ARG
    vol = adgi.volume_for_scene(sc, max_rays=4096, max_chains=64)
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_chains(0, 64, 40, 0)  # 2 * 64 * 39 rays > 4096
    assert e.value.status == adgi.ADGI_ERR_BUDGET
    for bad in ((65, 8, 1), (16, 1, 0), (16, 8, 7), (16, 300, 1)):
        with pytest.raises(adgi.AdgiError) as e:
            vol.update_chains(0, *bad)
        assert e.value.status == adgi.ADGI_ERR_INVALID_ARG, bad
    with pytest.raises(adgi.AdgiError):
        vol.update_chains(0, 16, 8, 1, sigma_pos=0.0)
    st = vol.update_chains(0, 64, 16, 0, sync=True)
    assert st["primary_rays"] == 2 * 64 * 15
    vol.destroy_volume()


def _dyn_run(sc, frames, tuning=None, vol=None, start=0):
    own = vol is None
    if own:
        vol = adgi.volume_for_scene(sc, max_rays=2 * 512 * 20 + sc.num_probes * 232, seed=6, max_chains=512)
    if tuning:
        vol.set_tuning(**tuning)
    for f in range(start, start + frames):
        vol.update_scene(sc.positions_at(f), light_pos=sc.light_positions(f),
                         light_intensity=sc.light_intensity, sky=sc.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, sc.anim_vertices))
        if f < 1:
            vol.update_probes(f, adaptive=False, n_uniform=32, sync=True)
        else:
            vol.update_chains(f, 512, 24, 3, sync=True, dyn_chains=128, dyn_steps=12, dyn_burn_in=2)
    rb = vol.read_probes()
    if own:
        vol.destroy_volume()
    return rb


def _same_dyn(a, b):
    _same_chain(a, b)
    for k in ("dyn_mark", "dyn_target", "dyn_state", "dyn_ray_offsets"):
        assert np.array_equal(a[k], b[k]), (k, int(np.count_nonzero(a[k] != b[k])))


@pytest.mark.parametrize("tuning", [{"use_graph": 0}, {"chain_lanes": 1}, {"persistent": 0}, {"bvh_width": 4}])
def test_dynamic_chain_launch_shape_does_not_change_results(tuning):
    sc = _small_field()
    a = _dyn_run(sc, 5)
    assert a["dyn_mark"].sum() > 0 and a["num_dyn_rays"] > 0
    _same_dyn(a, _dyn_run(sc, 5, tuning=tuning))


def test_dynamic_chain_snapshot_resumes_bit_identically():
    sc = _small_field()
    ref = _dyn_run(sc, 6)
    vol = adgi.volume_for_scene(sc, max_rays=2 * 512 * 20 + sc.num_probes * 232, seed=6, max_chains=512)
    _dyn_run(sc, 3, vol=vol)
    snap = vol.save_state()
    vol.destroy_volume()
    vol2 = adgi.volume_for_scene(sc, max_rays=2 * 512 * 20 + sc.num_probes * 232, seed=6, max_chains=512)
    vol2.restore_state(snap)
    got = _dyn_run(sc, 3, vol=vol2, start=3)
    vol2.destroy_volume()
    _same_dyn(ref, got)


def test_dynamic_chain_capacity_check():
    sc = scenes.box_field(seed=scenes.SEED_BASE + 211, lattice=16, dims=(8, 2, 8), n_lights=1, frames=2)
    vol = adgi.volume_for_scene(sc, max_rays=4096, max_chains=64)
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_chains(0, 16, 8, 1, dyn_chains=64, dyn_steps=16, dyn_burn_in=1)
    assert e.value.status == adgi.ADGI_ERR_BUDGET
    with pytest.raises(adgi.AdgiError) as e:
        vol.update_chains(0, 16, 8, 1, dyn_chains=65, dyn_steps=16, dyn_burn_in=1)
    assert e.value.status == adgi.ADGI_ERR_INVALID_ARG
    vol.destroy_volume()


@pytest.mark.parametrize("tuning", [{"use_graph": 0}, {"blend_blocks_per_cu": 4}, {"bvh_width": 4}])
def test_gather_launch_shape_does_not_change_results(tuning):
    sc = _small_field()

    def run(t):
        vol = adgi.volume_for_scene(sc, max_rays=sc.num_probes * 40, seed=3, blend_mode=adgi.ADGI_BLEND_GATHER)
        return _run(sc, 4, True, tuning=t, budget=sc.num_probes * 40, vol=vol)

    _same(run(None), run(tuning))


def test_gather_rejected_where_unsupported():
    sc = scenes.box_field(seed=scenes.SEED_BASE + 212, lattice=16, dims=(8, 2, 8), n_lights=1, frames=2)
    with pytest.raises(adgi.AdgiError):
        adgi.volume_for_scene(sc, max_rays=4096, storage=adgi.ADGI_PACKED, blend_mode=adgi.ADGI_BLEND_GATHER)
    vol = adgi.volume_for_scene(sc, max_rays=4096, blend_mode=adgi.ADGI_BLEND_GATHER, max_chains=16)
    with pytest.raises(adgi.AdgiError):
        vol.update_chains(0, 16, 8, 1)
    with pytest.raises(adgi.AdgiError):
        vol.set_tuning(blend_chunk=128)
    vol.update_probes(0, adaptive=False, n_uniform=16, sync=True)
    vol.destroy_volume()
