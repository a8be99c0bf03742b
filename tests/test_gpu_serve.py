"""Serving through the C ABI (needs an MI355X): many volumes under an HBM
budget that forces evictions; each stream's texels must equal, bit for bit,
those of the same stream run alone on a plain volume."""
import numpy as np
import pytest

import paper_2301_05125_amd as adgi
import scenes

pytestmark = pytest.mark.gpu

KEYS = ("irradiance", "depth", "irr_count", "depth_count", "rays_per_probe", "score")


def _streams():
    out = []
    for k, (lattice, dims, lights) in enumerate([(24, (8, 2, 8), 1), (40, (16, 4, 16), 2),
                                                 (32, (12, 3, 12), 3), (56, (16, 4, 16), 1),
                                                 (20, (8, 2, 8), 2), (48, (20, 5, 20), 3)]):
        sc = scenes.box_field(seed=scenes.SEED_BASE + 200 + k, lattice=lattice, dims=dims,
                              n_lights=lights, frames=8)
        out.append(sc)
    return out


def _alone(sc, frames, budget, seed):
    vol = adgi.volume_for_scene(sc, max_rays=budget, seed=seed)
    for f in range(frames):
        vol.update_scene(sc.positions, light_pos=sc.light_positions(f),
                         light_intensity=sc.light_intensity, sky=sc.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, 0))
        vol.update_probes(f, adaptive=True, budget=budget, n_min=8, n_max=2048, sync=True)
    rb = vol.read_probes()
    vol.destroy_volume()
    return rb


def test_serving_mix_equals_streams_alone():
    scs = _streams()
    srv = adgi.Server(hbm_budget_bytes=1 << 40, max_inflight=3)
    sids, budgets = [], []
    for k, sc in enumerate(scs):
        b = 48 * sc.num_probes
        sids.append(srv.add_stream(sc, budget=b, seed=100 + k))
        budgets.append(b)
    foot = [srv.stream_info(s)["footprint_bytes"] for s in sids]
    # about half of the total fits: admission has to evict
    srv.set_budget(max(max(foot), sum(foot) // 2))
    rng = np.random.Generator(np.random.PCG64(7))
    frames = [int(x) for x in rng.integers(3, 7, size=len(sids))]
    order = np.concatenate([np.full(n, s) for s, n in zip(sids, frames)])
    rng.shuffle(order)
    sent = [0] * len(sids)
    for s in order:
        srv.submit(int(s), scs[s].light_positions(sent[s]))
        sent[s] += 1
        srv.progress()
    srv.drain()
    assert srv.stats()["evictions"] > 0
    # one more frame for every stream: the evicted ones come back through
    # admission and restore their state
    for s in sids:
        srv.submit(int(s), scs[s].light_positions(sent[s]))
        sent[s] += 1
        frames[s] += 1
        srv.progress()
    srv.drain()
    st = srv.stats()
    print(st)
    assert st["completed"] == st["submitted"] == sum(frames)
    assert st["evictions"] > 0 and st["admissions"] > len(sids)
    assert st["peak_resident_bytes"] <= max(max(foot), sum(foot) // 2)
    assert st["primary_rays"] == sum(b * n for b, n in zip(budgets, frames))
    lat = srv.latencies()
    assert lat.size == sum(frames) and np.all(lat > 0)
    for k, s in enumerate(sids):
        mix = srv.read_stream(s)
        ref = _alone(scs[k], frames[k], budgets[k], 100 + k)
        for key in KEYS:
            assert np.array_equal(mix[key], ref[key]), (k, key)
    srv.destroy()


def test_serving_error_paths():
    sc = scenes.box_field(seed=scenes.SEED_BASE + 210, lattice=16, dims=(8, 2, 8), n_lights=1,
                          frames=2)
    srv = adgi.Server(hbm_budget_bytes=1 << 12, max_inflight=2)
    with pytest.raises(adgi.AdgiError) as e:
        srv.add_stream(sc, budget=16 * sc.num_probes)
    assert e.value.status == adgi.ADGI_ERR_OUT_OF_MEMORY
    srv.set_budget(1 << 34)
    sid = srv.add_stream(sc, budget=16 * sc.num_probes)
    with pytest.raises(adgi.AdgiError):
        srv.submit(sid + 5, sc.light_positions(0))
    with pytest.raises(adgi.AdgiError):
        srv.add_stream(sc, budget=4 * sc.num_probes)  # below P * n_min
    srv.submit(sid, sc.light_positions(0))
    srv.drain()
    assert srv.stats()["completed"] == 1
    srv.destroy()
