#!/usr/bin/env python
"""Probe-update benchmark on one MI355X: probe rays/s and p50/p99 update latency,
adaptive vs uniform, with rooflines of the two dominant kernels and the CPU
oracle timed beside it.

A step is one whole frame of the hot path on the 1M-triangle box field
(65,536 probes, 5% of the boxes animated, 3 moving lights): scene refit and
light update, pilot rays, change detection, budget allocation (B = 2^23,
8..2048 rays per probe), probe-ray trace with shadow rays, and the texel
blend. ``value`` is probe (primary) rays per second over the timed steps.
"""
from __future__ import annotations

import argparse
import faulthandler
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "probe rays/sec + p50/p99 probe-update ms/frame, adaptive vs uniform, 1 MI355X"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak of one MI355X in lane operations (an FMA is one operation):
# 157.3 TFLOP/s counts an FMA as two flops, i.e. 256 CUs x 128 lanes x 2.4 GHz.
# Non-packed VOP2 code reaches most of it (v_add_f32 with independent chains
# sustains 68 T ops/s), so the 64-lane-per-clock figure is not the ceiling.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# FP32 operations of the two traversal tests as written (adgi_device.hpp):
# slab test of one child box = 6 fma + 6 min/max + 6 min/max + 1 compare = 19,
# a BVH2 node visit tests two child boxes, a BVH4 visit four; Moller-Trumbore
# = 2 crosses (12), 4 dots (12), 3 subtractions, 2 sign products, 4 compares
# = 33.
OPS_PER_BOX = 19
OPS_PER_TRI = 33

WORKLOADS = {
    "box_field": dict(budget=1 << 23, n_min=8, n_max=2048, uniform_equal_b=128, uniform_equal_rays=136),
    "tunnel": dict(budget=1 << 19, n_min=32, n_max=1024, uniform_equal_b=256, uniform_equal_rays=264),
}


# committed counter summary of the blend kernel of each texel storage
BLEND_PROFILE = {"fp32": "blend_boxfield", "fp16": "blend_fp16_boxfield", "packed": "blend_packed_boxfield"}


def blend_bytes(P, R, storage):
    """Algorithmic HBM bytes of one blend launch: per probe read the interior
    texels (36 x 12 + 196 x 8 B FP32), write full tiles (64 x 12 + 256 x 8 B),
    read+write counts (2 x 232 B); FP16 halves the texel bytes; packed words
    (counts inside) read 232 x 4 B and write 320 x 4 B; 16 B per ray."""
    per_probe = {"fp32": 5280, "fp16": 2872, "packed": 2208}[storage]
    return P * per_probe + 16 * R


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2301_05125_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_profile(kernel_key, src_hash):
    """Counter figures from a committed rocprofv3 summary (HBM bytes per
    dispatch, VALU busy/utilisation), valid only while the kernel source is
    unchanged; {} otherwise."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_pmc.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != src_hash:
        return {}
    out = {"kernel_name": vals.get("kernel", "")}
    for key, name in (("hbm_bytes_per_dispatch", "traffic"), ("VALUBusy", "valu_busy_pct"),
                      ("VALUUtilization", "valu_utilization_pct"), ("kernel_trace_avg_us", "rocprof_avg_us")):
        try:
            out[name] = float(vals[key])
        except (KeyError, ValueError):
            pass
    return out


def profile_matches_width(kernel_name, width):
    """True if a profiled traversal kernel (template <kind, count, width 4>)
    is the variant of the given BVH width."""
    m = re.search(r"<\s*\d+\s*,\s*(true|false)\s*,\s*(true|false)\s*>", kernel_name)
    return bool(m) and m.group(2) == ("true" if width == 4 else "false")


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write), best of reps, GB/s."""
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del x, y
    return 2 * nbytes / (best * 1e-3) / 1e9


def light_frame(frame, period=60):
    """Lights go back and forth along their seeded paths."""
    f = frame % (2 * period)
    return f if f <= period else 2 * period - f


_POS = {}


def step_scene(vol, sc, frame, adgi):
    """Scene update of one step: animated vertex prefix and lights."""
    pos = _POS.get(id(sc))
    if pos is None:
        pos = _POS[id(sc)] = sc.positions.copy()
    sc.write_animated(frame, pos)
    vol.update_scene(pos, light_pos=sc.light_positions(light_frame(frame)),
                     light_intensity=sc.light_intensity, sky=sc.sky, mode=adgi.ADGI_SCENE_REFIT,
                     refit_range=(0, sc.anim_vertices))


def run_mode(vol, sc, adgi, torch, frame0, steps, warmup, latency_frames, **p):
    f = frame0
    for _ in range(warmup):
        step_scene(vol, sc, f, adgi)
        vol.update_probes(f, sync=False, **p)
        f += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_scene(vol, sc, f, adgi)
        vol.update_probes(f, sync=False, **p)
        f += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # latency: one synchronous frame at a time; the scene update before it is
    # timed on its own (host work + upload + refit, to device completion)
    host_ms, gpu_ms, rays, shadow, scene_ms, shadow_only = [], [], [], [], [], []
    for _ in range(latency_frames):
        torch.cuda.synchronize()
        a = time.perf_counter()
        step_scene(vol, sc, f, adgi)
        torch.cuda.synchronize()
        scene_ms.append((time.perf_counter() - a) * 1e3)
        a = time.perf_counter()
        st = vol.update_probes(f, sync=True, **p)
        host_ms.append((time.perf_counter() - a) * 1e3)
        gpu_ms.append(st["ms_total"])
        rays.append(st["primary_rays"])
        shadow.append(st["shadow_rays"] + st["pilot_rays"])
        shadow_only.append(st["shadow_rays"])
        f += 1
    return dict(seconds=t1 - t0, frames_end=f, host_ms=host_ms, gpu_ms=gpu_ms, scene_ms=scene_ms,
                rays_per_frame=sum(rays) / len(rays), extra_rays_per_frame=sum(shadow) / len(shadow),
                shadow_rays_per_frame=sum(shadow_only) / len(shadow_only))


def stage_times(vol, sc, adgi, frame0, frames, **p):
    """Per-kernel durations: eager launches with HIP events recorded between the
    kernels on the volume's own stream (the stream the kernels run on)."""
    tun = vol.get_tuning()
    vol.set_tuning(use_graph=0)
    acc = [0.0] * 8
    f = frame0
    for _ in range(frames):
        step_scene(vol, sc, f, adgi)
        st = vol.update_probes(f, sync=True, **p)
        for k in range(8):
            acc[k] += st["ms_stage"][k]
        f += 1
    vol.set_tuning(use_graph=tun["use_graph"])
    return [a / frames for a in acc], f


def run_config(adgi, torch, sc, cfg, storage_name, tuning, steps, warmup, latency_frames, uniform=()):
    """Adaptive frames of one workload (and uniform baselines of the given
    rays per probe on fresh volumes): throughput, latency, stage times and
    the blend's HBM roofline. tuning None: autotuned for this scene."""
    storage = {"fp32": adgi.ADGI_FP32, "fp16": adgi.ADGI_FP16, "packed": adgi.ADGI_PACKED}[storage_name]
    P = sc.num_probes
    max_rays = max([cfg["budget"]] + [P * n for n in uniform])
    ad = dict(adaptive=True, budget=cfg["budget"], n_min=cfg["n_min"], n_max=cfg["n_max"])
    vol = adgi.volume_for_scene(sc, storage=storage, max_rays=max_rays, seed=11)
    if tuning is None:
        tuning = vol.autotune(0, **ad)
    else:
        vol.set_tuning(**tuning)
    r = run_mode(vol, sc, adgi, torch, 0, steps, warmup, latency_frames, **ad)
    stages, _ = stage_times(vol, sc, adgi, r["frames_end"], 5, **ad)
    vol.destroy_volume()
    R = r["rays_per_frame"]
    bbytes = blend_bytes(P, R, storage_name)
    gbs = bbytes / (stages[5] * 1e-3) / 1e9
    out = {"workload": f"{sc.name}: {sc.num_triangles} triangles, {P} probes "
                       f"{tuple(int(x) for x in sc.grid_dims)}, adaptive B={cfg['budget']} "
                       f"n in [{cfg['n_min']},{cfg['n_max']}], texels {storage_name}",
           "tuning": tuning,
           "adaptive": {"rays_per_s": R * steps / r["seconds"], "ms_per_step": r["seconds"] / steps * 1e3,
                        "probe_updates_per_s": P * steps / r["seconds"],
                        "p50_ms": pct(r["host_ms"], 50), "p99_ms": pct(r["host_ms"], 99),
                        "gpu_p50_ms": pct(r["gpu_ms"], 50), "gpu_p99_ms": pct(r["gpu_ms"], 99),
                        "stage_ms": dict(zip(["setup", "pilot_trace", "detect", "allocate", "probe_trace",
                                              "blend", "probe_trace_hit", "probe_trace_shade"], stages))},
           "roofline_blend": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS, "ms": stages[5], "algorithmic_bytes": bbytes,
                              "traffic": read_profile(BLEND_PROFILE[storage_name],
                                                      source_hash("blend.hip", "adgi_device.hpp")).get("traffic"),
                              "target_ms_at_half_peak": bbytes / (0.5 * HBM_PEAK_GBS * 1e9) * 1e3}}
    for n in uniform:
        v2 = adgi.volume_for_scene(sc, storage=storage, max_rays=max_rays, seed=11)
        v2.set_tuning(**tuning)
        ru = run_mode(v2, sc, adgi, torch, 0, steps, warmup, latency_frames, adaptive=False, n_uniform=n)
        v2.destroy_volume()
        out[f"uniform_{n}"] = {"rays_per_probe": n, "rays_per_s": P * n * steps / ru["seconds"],
                               "ms_per_step": ru["seconds"] / steps * 1e3,
                               "p50_ms": pct(ru["host_ms"], 50), "p99_ms": pct(ru["host_ms"], 99),
                               "gpu_p50_ms": pct(ru["gpu_ms"], 50), "gpu_p99_ms": pct(ru["gpu_ms"], 99)}
    return out


# Chain frames on the same scene: the paper's 4096 static chains (about 64
# used samples each, Sec. 5), and as many chains as probes,
# which traces the adaptive budget B = 2^23 (two rays per sample).
CHAIN_CONFIGS = {
    "paper_4096_chains": dict(chains=4096, steps=80, burn_in=15),
    "equal_budget": dict(chains=65536, steps=80, burn_in=15),
    # the paper's 4096 static + 1024 dynamic chains (Sec. 5)
    "paper_static_dynamic": dict(chains=4096, steps=80, burn_in=15, dyn_chains=1024, dyn_steps=8,
                                 dyn_burn_in=3),
}
CHAIN_STAGES = ["setup", "pilot_trace", "chains_and_sort", "blend_order", "sample_trace", "blend"]


def run_chains(adgi, torch, sc, storage, tuning, steps, warmup, latency_frames, chains, steps_per_chain,
               burn_in, dyn_chains=0, dyn_steps=0, dyn_burn_in=0):
    """Chain frames: two warm uniform frames give the guide an irradiance,
    then `warmup` untimed and `steps` timed chain frames (scene update
    included, as in the budgeted steps), then synchronous frames for latency
    (captured frame graphs, as in the timed frames), then a few eager frames
    with stage events between the kernels for the per-stage times."""
    P = sc.num_probes
    S = steps_per_chain - burn_in - 1
    Sd = dyn_steps - dyn_burn_in - 1 if dyn_chains else 0
    pd = [(int(x) + 2) // 3 for x in sc.grid_dims]
    dyn_cap = min(P * 232, 27 * 34 * min(8 * pd[0] * pd[1] * pd[2], dyn_chains * Sd)) if dyn_chains else 0
    vol = adgi.volume_for_scene(sc, storage=storage, max_rays=max(2 * chains * S + dyn_cap, P * 32), seed=11,
                                max_chains=max(chains, dyn_chains))
    vol.set_tuning(**tuning)
    kw = dict(chains=chains, steps=steps_per_chain, burn_in=burn_in, dyn_chains=dyn_chains, dyn_steps=dyn_steps,
              dyn_burn_in=dyn_burn_in)
    f = 0
    for _ in range(2):
        step_scene(vol, sc, f, adgi)
        vol.update_probes(f, adaptive=False, n_uniform=32, sync=False)
        f += 1
    for _ in range(warmup):
        step_scene(vol, sc, f, adgi)
        vol.update_chains(f, sync=False, **kw)
        f += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_scene(vol, sc, f, adgi)
        vol.update_chains(f, sync=False, **kw)
        f += 1
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    host_ms, gpu_ms, stage, rays_seen, marks = [], [], [0.0] * 6, [], []
    for _ in range(latency_frames):
        step_scene(vol, sc, f, adgi)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = vol.update_chains(f, sync=True, **kw)
        host_ms.append((time.perf_counter() - a) * 1e3)
        gpu_ms.append(st["ms_total"])
        rays_seen.append(st["primary_rays"])
        if dyn_chains:
            marks.append(int(vol.read_probes(texels=False)["dyn_mark"].sum()))
        f += 1
    tun = vol.get_tuning()
    vol.set_tuning(use_graph=0)
    stage_frames = 6  # both frame parities
    for _ in range(stage_frames):
        step_scene(vol, sc, f, adgi)
        st = vol.update_chains(f, sync=True, **kw)
        for k in range(6):
            stage[k] += st["ms_stage"][k] / stage_frames
        f += 1
    vol.set_tuning(use_graph=tun["use_graph"])
    tw = vol.measure_chain_trace_work(f, **kw)
    rb = vol.read_probes(texels=False)
    n = rb["rays_per_probe"]
    vol.destroy_volume()
    # rays per frame: 2 per static sample plus the dynamic texel-centre rays
    # (measured on the synchronous frames; the timed frames trace as many)
    rays = sum(rays_seen) / len(rays_seen)
    trace_ms = stage[4]
    nr = max(tw["primary_rays"] + tw["shadow_rays"], 1)
    return {"chains": chains, "steps": steps_per_chain, "burn_in": burn_in, "samples_per_frame": chains * S,
            "rays_per_frame": rays, "rays_per_s": rays * steps / seconds,
            "ms_per_step": seconds / steps * 1e3,
            "p50_ms": pct(host_ms, 50), "p99_ms": pct(host_ms, 99),
            "gpu_p50_ms": pct(gpu_ms, 50), "gpu_p99_ms": pct(gpu_ms, 99),
            "stage_ms": dict(zip(CHAIN_STAGES, stage)),
            "sample_trace_mrays_per_s_incl_shadow": nr / (trace_ms * 1e-3) / 1e6 if trace_ms else None,
            "sample_trace_tops": (tw["box_tests"] * OPS_PER_BOX + tw["tri_tests"] * OPS_PER_TRI)
            / (trace_ms * 1e-3) / 1e12 if trace_ms else None,
            "probes_with_samples": int((n > 0).sum()), "max_samples_per_probe": int(n.max()),
            **({"dyn_chains": dyn_chains, "dyn_steps": dyn_steps, "dyn_burn_in": dyn_burn_in,
                "marked_proxy_octants_per_frame": sum(marks) / len(marks),
                "dynamic_rays_per_frame": rays - 2 * chains * S} if dyn_chains else {})}


def run_quality(adgi, torch, sc, cfg, tuning, frames=40, every=8, ref_rays=2304):
    """Texel error of the samplers at equal rays per frame against a converged
    reference (the paper's protocol for its reference renderer, Sec. 5: the
    texels are cleared every frame and take a true average, here of
    ref_rays = 64 x 36 spherical-Fibonacci rays per probe, hysteresis close to
    1 so that a = 1/(N+1)). Every `every` frames of the animated scene the
    reference is rebuilt at that frame and each sampler's irradiance
    luminance is compared texel by texel: RMSE and mean absolute error
    relative to the mean reference luminance, over all probes and over the
    probes whose reference changed most since the previous checkpoint (the
    top 10%). A second reference with other rays gives the reference's own
    noise on the same scale."""
    import numpy as np
    P = sc.num_probes
    B = cfg["budget"]
    contenders = {
        "adaptive": dict(kind="adaptive"),
        "adaptive_gather": dict(kind="adaptive", gather=True),
        "uniform": dict(kind="uniform", n=B // P),
        "chains": dict(kind="chains", chains=B // 128, steps=80, burn_in=15),
    }
    vols = {}
    for name, c in contenders.items():
        if c["kind"] == "chains":
            v = adgi.volume_for_scene(sc, max_rays=B + P * 64, seed=11, max_chains=c["chains"])
        else:
            v = adgi.volume_for_scene(sc, max_rays=max(B, P * c.get("n", 0)), seed=11,
                                      blend_mode=adgi.ADGI_BLEND_GATHER if c.get("gather") else adgi.ADGI_BLEND_SAMPLE)
        t = dict(tuning)
        if c.get("gather"):
            t["blend_chunk"] = 0
        v.set_tuning(**t)
        vols[name] = v
    ref = adgi.volume_for_scene(sc, max_rays=P * ref_rays, seed=12, hysteresis=0.99999)
    ref2 = adgi.volume_for_scene(sc, max_rays=P * ref_rays, seed=13, hysteresis=0.99999)
    blank = ref.save_state()

    def lum(rb):
        irr = rb["irradiance"][:, 1:-1, 1:-1, :].astype(np.float64)
        return 0.2126 * irr[..., 0] + 0.7152 * irr[..., 1] + 0.0722 * irr[..., 2]

    out = {name: [] for name in list(contenders) + ["reference_noise"]}
    prev_ref = None
    rays = {name: 0 for name in contenders}
    for f in range(frames):
        for name, v in vols.items():
            step_scene(v, sc, f, adgi)
            c = contenders[name]
            if c["kind"] == "adaptive":
                st = v.update_probes(f, adaptive=True, budget=B, n_min=cfg["n_min"], n_max=cfg["n_max"], sync=True)
            elif c["kind"] == "uniform" or f < 2:
                st = v.update_probes(f, adaptive=False, n_uniform=c.get("n", 32), sync=True)
            else:
                st = v.update_chains(f, c["chains"], c["steps"], c["burn_in"], sync=True)
            rays[name] += st["primary_rays"]
        if f % every != every - 1:
            continue
        refs = []
        for rv in (ref, ref2):
            rv.restore_state(blank)
            step_scene(rv, sc, f, adgi)
            rv.update_probes(f, adaptive=False, n_uniform=ref_rays, sync=True)
            refs.append(lum(rv.read_probes()))
        lr = refs[0]
        mean = float(lr.mean())
        changed = None
        if prev_ref is not None:
            d = np.abs(lr - prev_ref).reshape(P, -1).mean(axis=1)
            changed = d >= np.quantile(d, 0.9)
        prev_ref = lr
        for name in out:
            got = refs[1] if name == "reference_noise" else lum(vols[name].read_probes())
            e = (got - lr).reshape(P, -1)
            row = {"frame": f, "rmse_rel": float(np.sqrt(np.mean(e * e)) / mean),
                   "mae_rel": float(np.mean(np.abs(e)) / mean)}
            if changed is not None:
                row["rmse_rel_changed"] = float(np.sqrt(np.mean(e[changed] ** 2)) / mean)
                row["mae_rel_changed"] = float(np.mean(np.abs(e[changed])) / mean)
            out[name].append(row)
        print(f"[bench] quality frame {f}: mae " + ", ".join(
            f"{n} {out[n][-1]['mae_rel']:.4f}" for n in out), file=sys.stderr, flush=True)
    for v in list(vols.values()) + [ref, ref2]:
        v.destroy_volume()
    summary = {}
    for name in out:
        rows = out[name][1:]  # after the first checkpoint the caches have history
        summary[name] = {"rays_per_frame": rays[name] / frames if name in rays else ref_rays * P,
                         **{f"{m}_mean": float(np.mean([r[m] for r in rows]))
                            for m in ("rmse_rel", "mae_rel", "rmse_rel_changed", "mae_rel_changed")},
                         "checkpoints": out[name]}
    return {"reference": f"cleared every checkpoint, true average of {ref_rays} rays per probe",
            "frames": frames, "every": every, "samplers": summary}


def run_colour_slices(adgi, torch, n=256, scales=(1 / 256, 1 / 64, 1 / 16, 1 / 4, 1.0, 4.0, 8.0)):
    """The packed irradiance encoding (R9 G9 B8, log, rounded down; through
    the library's own encoder, adgi_pack_channel) against FP16 storage
    (round to nearest) on slices of RGB space across the dynamic range, each
    against the FP32 colours: at intensity scale s, the n x n slice
    s (r, g, b0) over r, g in [0, 1] for b0 in {0, 1/2, 1}, and likewise
    s (r0, g, b) for r0 in {0, 1/2, 1}. Errors as the paper's encoding
    comparison reports them: luminance error, the r.m.s. difference of the
    Rec. 709 luminance maps (also relative to the mean reference luminance),
    and colour correlation, the normalised dot product of the flattened
    colour maps."""
    dev = torch.device("cuda")
    t = torch.linspace(0.0, 1.0, n, device=dev, dtype=torch.float32)
    a, b = torch.meshgrid(t, t, indexing="ij")
    w = torch.tensor([0.2126, 0.7152, 0.0722], device=dev, dtype=torch.float64)
    rows = {"packed_r9g9b8": [], "fp16": []}
    for s in scales:
        acc = {k: {"se": 0.0, "lum": 0.0, "dot": 0.0, "n_enc": 0.0, "n_ref": 0.0, "count": 0} for k in rows}
        for fixed in (0.0, 0.5, 1.0):
            c = torch.full_like(a, fixed)
            for rgb in (torch.stack([a, b, c], -1), torch.stack([c, a, b], -1)):
                ref = (rgb * s).contiguous()
                _, d_rg = adgi.pack_channel(ref[..., :2].contiguous(), adgi.ADGI_PACK_RG9)
                _, d_b = adgi.pack_channel(ref[..., 2].contiguous(), adgi.ADGI_PACK_B8)
                enc = {"packed_r9g9b8": torch.cat([d_rg, d_b[..., None]], -1),
                       "fp16": ref.half().float()}
                r64 = ref.double()
                y_ref = r64 @ w
                for k, e in enc.items():
                    e64 = e.double()
                    dy = e64 @ w - y_ref
                    A = acc[k]
                    A["se"] += float((dy * dy).sum())
                    A["lum"] += float(y_ref.sum())
                    A["dot"] += float((e64 * r64).sum())
                    A["n_enc"] += float((e64 * e64).sum())
                    A["n_ref"] += float((r64 * r64).sum())
                    A["count"] += int(dy.numel())
        for k, A in acc.items():
            rms = (A["se"] / A["count"]) ** 0.5
            rows[k].append({"scale": s, "lum_rms": rms, "lum_rms_rel": rms / (A["lum"] / A["count"]),
                            "colour_correlation": A["dot"] / ((A["n_enc"] * A["n_ref"]) ** 0.5)})
    torch.cuda.synchronize()
    return {"slices": f"{n}x{n} RGB slices s(r, g, b0) and s(r0, g, b), b0, r0 in {{0, 1/2, 1}}, "
                      f"scales {list(scales)} (the packed range ends at (e^5 - 1)/15 = 9.83)",
            "reference": "FP32 colours", **rows}


def cpu_baseline(sc, budget, n_min, n_max, sample_probes=4096, frames=2):
    """The oracle as it stands, on the host cores, on a bounded sample of the
    adaptive frame: the scene update, all pilot rays, detection and allocation
    of the whole grid, and the probe rays of ``sample_probes`` sampled probes.
    The probe-ray phase is scaled from the sample to all B rays of the frame;
    the whole-grid phases are timed in full."""
    import oracle
    import scenes as S
    probes = S.sample_probes(sc.num_probes, sample_probes)
    vol = oracle.OracleVolume(sc, seed=7, probes=probes)
    fixed = probes_s = 0.0
    sample_rays = full_rays = 0
    t0 = time.perf_counter()
    for f in range(frames):
        out = vol.update(f, adaptive=True, budget=budget, n_min=n_min, n_max=n_max)
        sec = out["seconds"]
        fixed += sec["scene"] + sec["pilots"] + sec["detect_allocate"]
        probes_s += sec["probes"]
        sample_rays += out["counts"]["rays"]
        full_rays += int(out["n"].sum())
    wall = time.perf_counter() - t0
    frame_s = (fixed + probes_s * full_rays / max(sample_rays, 1)) / frames
    return {"value": full_rays / frames / frame_s, "unit": "rays/s",
            "cores": int(oracle.lib().orc_num_threads()), "kind": "oracle",
            "sample": f"{frames} adaptive frames of the box field: scene update, all "
                      f"{8 * sc.num_probes} pilot rays (+ shadow rays), detection and allocation "
                      f"of B={budget} timed in full ({fixed:.1f} s); probe rays (+ shadow rays) of "
                      f"{len(probes)} sampled probes, {sample_rays} rays in {probes_s:.1f} s, "
                      f"scaled to all {full_rays} probe rays; {wall:.1f} s of oracle work "
                      f"(BVH build untimed)",
            "sampled_probe_rays_per_s": sample_rays / max(probes_s, 1e-9),
            "extrapolated_ms_per_frame": frame_s * 1e3,
            "seconds": wall,
            "host": host_info(),
            "box_field_fp16_storage": cpu_box_field_variants(oracle, sc, probes, budget, n_min, n_max),
            "other_workloads": cpu_small_workloads(oracle)}


def cpu_box_field_variants(oracle, sc, probes, budget, n_min, n_max):
    """The box field's FP16-storage frame (the texels rounded to binary16 after
    every update, as the GPU's FP16 storage) on all threads, and its probe rays
    on one thread, each on a bounded sample of probes: 1,024 probes for two
    adaptive FP16 frames (probe-ray phase only, scaled to all B rays), 256
    probes for one uniform frame of 128 rays per probe on one thread."""
    out = {}
    v16 = oracle.OracleVolume(sc, seed=7, fp16=True, probes=probes[:1024])
    probes_s = 0.0
    sample_rays = full_rays = 0
    for f in range(2):
        o = v16.update(f, adaptive=True, budget=budget, n_min=n_min, n_max=n_max)
        probes_s += o["seconds"]["probes"]
        sample_rays += o["counts"]["rays"]
        full_rays += int(o["n"].sum())
    out["fp16_probe_rays_per_s"] = sample_rays / max(probes_s, 1e-9)
    out["fp16_sample"] = f"probe rays of 1024 sampled probes over 2 adaptive frames, {sample_rays} rays"
    v1 = oracle.OracleVolume(sc, seed=7, probes=probes[:256])
    nthreads = int(oracle.lib().orc_num_threads())
    oracle.lib().orc_set_threads(1)
    try:
        o = v1.update(0, adaptive=False, n_uniform=128)
    finally:
        oracle.lib().orc_set_threads(nthreads)
    out["one_thread_probe_rays_per_s"] = o["counts"]["rays"] / max(o["seconds"]["probes"], 1e-9)
    out["one_thread_sample"] = f"probe rays of 256 sampled probes, 128 each, one thread, {o['counts']['rays']} rays"
    return out


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_small_workloads(oracle):
    """The Cornell room (uniform, 64 rays/probe) and the tunnel (adaptive,
    B = 2^19) as full oracle frames on all threads, and the tunnel's probe
    rays on one thread (a bounded sample of its probes)."""
    import scenes as S
    out = {}
    sc = S.cornell()
    vol = oracle.OracleVolume(sc, seed=7)
    t0 = time.perf_counter()
    rays = 0
    for f in range(2):
        rays += vol.update(f, adaptive=False, n_uniform=64)["counts"]["rays"]
    dt = time.perf_counter() - t0
    out["cornell_full_frame"] = {"rays_per_s": rays / dt, "ms_per_frame": dt / 2 * 1e3}
    sc = S.tunnel()
    vol = oracle.OracleVolume(sc, seed=7)
    frame_s = []
    rays = 0
    for f in range(2):
        o = vol.update(f, adaptive=True, budget=1 << 19, n_min=32, n_max=1024)
        frame_s.append(sum(o["seconds"].values()))
        rays += o["counts"]["rays"]
    out["tunnel_full_frame"] = {"rays_per_s": rays / sum(frame_s),
                                "ms_per_frame": sum(frame_s) / 2 * 1e3}
    probes = S.sample_probes(sc.num_probes, 128)
    vol = oracle.OracleVolume(sc, seed=7, probes=probes)
    nthreads = int(oracle.lib().orc_num_threads())
    oracle.lib().orc_set_threads(1)
    try:
        o = vol.update(0, adaptive=True, budget=1 << 19, n_min=32, n_max=1024)
    finally:
        oracle.lib().orc_set_threads(nthreads)
    out["tunnel_one_thread"] = {"rays_per_s": o["counts"]["rays"] / max(o["seconds"]["probes"], 1e-9),
                                "sample": f"probe rays of 128 sampled probes, {o['counts']['rays']} rays"}
    return out


def run_serving_child(duration_s):
    """The serving mix in a process of its own: a failure there is reported
    in its place ({"error": ...}, with the end of the child's stderr) and does
    not take the main measurement with it; main() also lists it under the
    line's top-level "errors"."""
    import subprocess
    try:
        # ADGI_CRASH_TRACE: a fault there prints the library's native stack too
        r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--serve-only",
                            "--serve-seconds", str(duration_s)], capture_output=True, text=True,
                           timeout=240 + 40 * duration_s, env=dict(os.environ, ADGI_CRASH_TRACE="1"))
    except subprocess.TimeoutExpired:
        return {"error": "serving process timed out"}
    sys.stderr.write(r.stderr[-3000:])
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"serving process exited with status {r.returncode}",
                "stderr_tail": r.stderr[-1500:]}
    return json.loads(lines[-1])


def serve_phase(srv, sids, streams, scale, duration_s, nframe):
    """One serving phase: every stream's Poisson arrivals with its rate times
    ``scale`` (the seeded arrival times divided by scale) for duration_s, then
    a drain. Latencies, rays and device busy time are this phase's share of
    the server's running totals."""
    import numpy as np
    lat0 = len(srv.latencies())
    st0 = srv.stats()
    events = sorted((float(t) / scale, k) for k, st in enumerate(streams) for t in st.arrivals
                    if float(t) / scale < duration_s)
    start = srv.now_ns() + 20_000_000
    for t, k in events:
        target = start + int(t * 1e9)
        while srv.now_ns() < target:
            srv.progress()
        srv.submit(sids[k], streams[k].scene.light_positions(nframe[k] % streams[k].scene.frames),
                   arrival_ns=target)
        nframe[k] += 1
        srv.progress()
    srv.drain()
    span = (srv.now_ns() - start) * 1e-9
    st1 = srv.stats()
    lat = srv.latencies()[lat0:]
    rays = st1["primary_rays"] - st0["primary_rays"]
    offered = sum(s.rate_hz * scale * s.budget for s in streams)
    return {"rate_scale": scale, "offered_rays_per_s": offered, "requests": len(events),
            "completed": int(st1["completed"] - st0["completed"]),
            "rays_per_s": rays / max(span, 1e-9),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(np.mean(lat)) if len(lat) else None,
            "max_ms": float(np.max(lat)) if len(lat) else None,
            "span_s": span,
            "device_overlap": (st1["device_busy_ms"] - st0["device_busy_ms"]) * 1e-3 / max(span, 1e-9),
            "admissions": int(st1["admissions"] - st0["admissions"]),
            "evictions": int(st1["evictions"] - st0["evictions"])}


def run_serving(adgi, duration_s=10.0, budget_frac=0.6, max_inflight=8, sweep=(0.7, 0.5)):
    """Serving mix: 32 streams (box fields of 10k-500k triangles, 512-32768
    probes, B = 128 rays per probe), Poisson arrivals at 30-120 Hz each, for
    duration_s of wall time, under an HBM admission budget of budget_frac of
    the streams' summed device footprints. First the mix as drawn (it offers
    more rays than the GPU completes: an overload, whose latencies measure
    queue growth), then the same arrival processes slowed so that they offer
    the given fractions of the throughput the overload phase completed.
    device_overlap is the mean number of frames on the device at once."""
    import scenes
    streams = scenes.serving_streams(duration_s=duration_s)
    srv = adgi.Server(hbm_budget_bytes=1 << 40, max_inflight=max_inflight)
    t0 = time.perf_counter()
    sids = [srv.add_stream(st.scene, budget=st.budget, seed=1000 + k) for k, st in enumerate(streams)]
    setup_s = time.perf_counter() - t0
    foot = [srv.stream_info(sid)["footprint_bytes"] for sid in sids]
    budget = max(int(budget_frac * sum(foot)), max(foot))
    srv.set_budget(budget)
    print(f"[bench] serving: {len(sids)} streams added in {setup_s:.1f}s, footprints "
          f"{sum(foot) / 2**30:.2f} GiB, budget {budget / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    nframe = [0] * len(streams)
    over = serve_phase(srv, sids, streams, 1.0, duration_s, nframe)
    print(f"[bench] serving overload phase: {over['rays_per_s'] / 1e9:.2f} G rays/s of "
          f"{over['offered_rays_per_s'] / 1e9:.2f} offered", file=sys.stderr, flush=True)
    phases = []
    for frac in sweep:
        scale = min(1.0, frac * over["rays_per_s"] / over["offered_rays_per_s"])
        ph = serve_phase(srv, sids, streams, scale, duration_s, nframe)
        ph["fraction_of_capacity"] = frac
        phases.append(ph)
        print(f"[bench] serving at {frac:.2f} of capacity: p50 {ph['p50_ms']:.1f} ms, "
              f"p99 {ph['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    out = {"streams": len(sids), "duration_s": duration_s, "overload": over, "below_capacity": phases,
           "hbm_budget_bytes": budget, "sum_footprint_bytes": sum(foot),
           "peak_resident_bytes": srv.stats()["peak_resident_bytes"], "max_inflight": max_inflight,
           "setup_s": setup_s, "triangles": [int(s.scene.num_triangles) for s in streams],
           "probes": [int(s.scene.num_probes) for s in streams]}
    srv.destroy()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="box_field", choices=sorted(WORKLOADS))
    ap.add_argument("--latency-frames", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "packed"])
    ap.add_argument("--tuning", default=None,
                    help="JSON launch tuning to use instead of the autotuner")
    ap.add_argument("--skip-uniform", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the FP16-storage box field and the tunnel (adaptive vs uniform)")
    ap.add_argument("--no-serve", action="store_true", help="skip the 32-stream serving mix")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving mix and print its JSON (the bench runs it so, as a child)")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the texel error against a converged reference (adaptive vs uniform vs chains)")
    ap.add_argument("--chains", default=",".join(CHAIN_CONFIGS),
                    help="comma-separated chain-frame configurations to run (none: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    faulthandler.enable()  # a crash prints the Python stack of every thread
    errors = []
    if args.serve_only:
        import torch
        import paper_2301_05125_amd as adgi
        torch.cuda.set_device(0)
        print(json.dumps(run_serving(adgi, duration_s=args.serve_seconds)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2301_05125_amd as adgi
    import scenes

    torch.cuda.set_device(0)
    cfg = WORKLOADS[args.workload]
    sc = scenes.box_field() if args.workload == "box_field" else scenes.tunnel()
    sc.frames = 61  # light_frame() walks frames 0..60 back and forth
    storage = {"fp32": adgi.ADGI_FP32, "fp16": adgi.ADGI_FP16, "packed": adgi.ADGI_PACKED}[args.storage]
    P = sc.num_probes
    max_rays = max(cfg["budget"], P * cfg["uniform_equal_rays"])
    print(f"[bench] workload={args.workload} P={P} tris={sc.num_triangles} B={cfg['budget']}",
          file=sys.stderr, flush=True)
    t = time.perf_counter()
    vol = adgi.volume_for_scene(sc, storage=storage, max_rays=max_rays, seed=11)
    build_s = time.perf_counter() - t
    ad = dict(adaptive=True, budget=cfg["budget"], n_min=cfg["n_min"], n_max=cfg["n_max"])
    tuning = vol.get_tuning()
    if args.tuning:
        vol.set_tuning(**json.loads(args.tuning))
        tuning = vol.get_tuning()
    elif not args.no_autotune:
        tuning = vol.autotune(0, **ad)
    print(f"[bench] scene build {build_s:.2f}s tuning={tuning}", file=sys.stderr, flush=True)

    res_a = run_mode(vol, sc, adgi, torch, 0, args.steps, args.warmup, args.latency_frames, **ad)
    print(f"[bench] adaptive done {res_a['seconds']:.3f}s", file=sys.stderr, flush=True)
    stages_a, fnext = stage_times(vol, sc, adgi, res_a["frames_end"], 5, **ad)
    tw = vol.measure_trace_work(fnext, **ad)

    # uniform baselines on fresh volumes (same scene, same tuning)
    uni = {}
    for name, n in (() if args.skip_uniform else
                    (("uniform_equal_budget", cfg["uniform_equal_b"]),
                     ("uniform_equal_traced", cfg["uniform_equal_rays"]))):
        v2 = adgi.volume_for_scene(sc, storage=storage, max_rays=max_rays, seed=11)
        v2.set_tuning(**tuning)
        r = run_mode(v2, sc, adgi, torch, 0, args.steps, args.warmup, args.latency_frames,
                     adaptive=False, n_uniform=n)
        uni[name] = dict(
            rays_per_probe=n,
            rays_per_s=P * n * args.steps / r["seconds"],
            ms_per_step=r["seconds"] / args.steps * 1e3,
            p50_ms=pct(r["host_ms"], 50), p99_ms=pct(r["host_ms"], 99),
            gpu_p50_ms=pct(r["gpu_ms"], 50), gpu_p99_ms=pct(r["gpu_ms"], 99))
        v2.destroy_volume()
        print(f"[bench] {name} done", file=sys.stderr, flush=True)

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")  # 256 MiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    copy_gbs = copy_bandwidth(torch)

    R = res_a["rays_per_frame"]
    value = R * args.steps / res_a["seconds"]
    ms_step = res_a["seconds"] / args.steps * 1e3
    trace_ms, blend_ms = stages_a[4], stages_a[5]
    bbytes = blend_bytes(P, R, args.storage)
    blend_gbs = bbytes / (blend_ms * 1e-3) / 1e9
    h_trace = source_hash("trace.hip", "adgi_device.hpp", "adgi_layout.hpp", "bvh_build.cpp")
    h_blend = source_hash("blend.hip", "adgi_device.hpp")
    prof_blend = read_profile(BLEND_PROFILE[args.storage], h_blend)
    width = 4 if tuning.get("bvh_width") == 4 else 2

    def trace_roof(kernel, ms, nodes, boxes, tris, rays, prof_key):
        """ALU roofline of one traversal kernel: its slab and triangle tests
        (counted by the work-counting run; empty BVH4 child slots excluded)
        over its eager duration."""
        ops = boxes * OPS_PER_BOX + tris * OPS_PER_TRI
        tops = ops / (ms * 1e-3) / 1e12 if ms else 0.0
        prof = read_profile(prof_key, h_trace)
        # the counters belong to one traversal variant (<kind, count, width 4>)
        if not profile_matches_width(prof.get("kernel_name", ""), width):
            prof = {}
        return {"bound": "alu", "kernel": "%s<primary, BVH%d>" % (kernel, width), "achieved": tops,
                "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s", "frac": tops / VALU_PEAK_TOPS,
                "traffic": prof.get("traffic"), "valu_busy_pct": prof.get("valu_busy_pct"),
                "valu_utilization_pct": prof.get("valu_utilization_pct"), "ms": ms, "rays": rays,
                "mrays_per_s": rays / (ms * 1e-3) / 1e6 if ms else None,
                "node_tests_per_ray": nodes / max(rays, 1), "box_tests_per_ray": boxes / max(rays, 1),
                "tri_tests_per_ray": tris / max(rays, 1), "bvh_width": width}

    roof_hit = trace_roof("trace_hit_kernel", stages_a[6], tw["node_tests"] - tw["shade_node_tests"],
                          tw["box_tests"] - tw["shade_box_tests"], tw["tri_tests"] - tw["shade_tri_tests"],
                          tw["primary_rays"], "trace_hit_boxfield")
    roof_shade = trace_roof("trace_shade_kernel", stages_a[7], tw["shade_node_tests"], tw["shade_box_tests"],
                            tw["shade_tri_tests"], tw["shadow_rays"], "trace_shade_boxfield")
    roof_blend = {"bound": "hbm", "kernel": "blend_kernel", "achieved": blend_gbs, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": blend_gbs / HBM_PEAK_GBS,
                  "traffic": prof_blend.get("traffic"), "ms": blend_ms,
                  "algorithmic_bytes": bbytes, "copy_gbs": copy_gbs, "frac_of_copy": blend_gbs / copy_gbs}
    dominant = max((roof_hit, roof_shade, roof_blend), key=lambda x: x["ms"])
    out = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {sc.num_triangles} triangles, {P} probes "
                               f"{tuple(int(x) for x in sc.grid_dims)}, adaptive B={cfg['budget']} "
                               f"n in [{cfg['n_min']},{cfg['n_max']}], 8x8 irradiance + 16x16 depth "
                               f"texels {args.storage}, 5% boxes refit per frame, "
                               f"{sc.num_lights} moving lights",
                   "parallelism": "1 GPU", "tuning": tuning},
        "adaptive": {"rays_per_s": value, "probe_updates_per_s": P * args.steps / res_a["seconds"],
                     "pilot_plus_shadow_rays_per_s": res_a["extra_rays_per_frame"] * args.steps / res_a["seconds"],
                     "shadow_rays_per_s": res_a["shadow_rays_per_frame"] * args.steps / res_a["seconds"],
                     "scene_update_p50_ms": pct(res_a["scene_ms"], 50),
                     "scene_update_p99_ms": pct(res_a["scene_ms"], 99),
                     "p50_ms": pct(res_a["host_ms"], 50), "p99_ms": pct(res_a["host_ms"], 99),
                     "gpu_p50_ms": pct(res_a["gpu_ms"], 50), "gpu_p99_ms": pct(res_a["gpu_ms"], 99),
                     "stage_ms": dict(zip(["setup", "pilot_trace", "detect", "allocate", "probe_trace",
                                           "blend", "probe_trace_hit", "probe_trace_shade"], stages_a))},
        **uni,
        "roofline": dominant,
        "roofline_trace_hit": roof_hit,
        "roofline_trace_shade": roof_shade,
        "trace": {"ms": trace_ms, "rays_incl_shadow": tw["primary_rays"] + tw["shadow_rays"],
                  "mrays_per_s_incl_shadow": (tw["primary_rays"] + tw["shadow_rays"]) / (trace_ms * 1e-3) / 1e6},
        "roofline_blend": roof_blend,
        "scene_build_s": build_s,
    }
    vol.destroy_volume()
    if not args.no_configs:
        # the FP16-storage variant of the same scene (texels stored as binary16,
        # FP32 arithmetic; launch shapes autotuned for it); its per-texel error
        # against the FP64 oracle is the parity suite's (box-field FP16
        # storage report)
        out["fp16_storage"] = run_config(adgi, torch, sc, cfg, "fp16", None, args.steps, args.warmup,
                                         min(args.latency_frames, 30))
        print("[bench] fp16 storage done", file=sys.stderr, flush=True)
        # the tunnel: adaptive B = 2^19 against uniform 256 (equal budget) and
        # 264 (equal traced rays, the budget plus the pilots) rays per probe
        tn = scenes.tunnel()
        tn.frames = 61
        tcfg = WORKLOADS["tunnel"]
        out["tunnel"] = run_config(adgi, torch, tn, tcfg, "fp32", None, args.steps, args.warmup,
                                   min(args.latency_frames, 30),
                                   uniform=(tcfg["uniform_equal_b"], tcfg["uniform_equal_rays"]))
        print("[bench] tunnel done", file=sys.stderr, flush=True)
    # DDGI's cosine-weighted gather in place of the per-sample update, same frames
    if not args.skip_uniform:
        vg = adgi.volume_for_scene(sc, storage=storage if args.storage != "packed" else adgi.ADGI_FP32,
                                   max_rays=max_rays, seed=11, blend_mode=adgi.ADGI_BLEND_GATHER)
        tg = dict(tuning)
        tg["blend_chunk"] = 0
        vg.set_tuning(**tg)
        rg = run_mode(vg, sc, adgi, torch, 0, args.steps, args.warmup, min(args.latency_frames, 20), **ad)
        stages_g, _ = stage_times(vg, sc, adgi, rg["frames_end"], 5, **ad)
        vg.destroy_volume()
        # per ray: 36 irradiance texels x 8 ops (dot 3, max 1, weight sum 1,
        # 3 fma) and 196 depth texels x 14 ops (dot 3, max 1, 7 multiplies for
        # the 50th power, weight sum 1, 2 fma), plus tau^2 once per ray
        gops = R * (36 * 8 + 196 * 14 + 1)
        out["gather_blend"] = {
            "rays_per_s": rg["rays_per_frame"] * args.steps / rg["seconds"],
            "ms_per_step": rg["seconds"] / args.steps * 1e3,
            "p50_ms": pct(rg["host_ms"], 50), "p99_ms": pct(rg["host_ms"], 99),
            "blend_ms": stages_g[5], "per_sample_blend_ms": blend_ms,
            "roofline": {"bound": "alu", "achieved": gops / (stages_g[5] * 1e-3) / 1e12, "peak": VALU_PEAK_TOPS,
                         "unit": "TFLOP/s", "frac": gops / (stages_g[5] * 1e-3) / 1e12 / VALU_PEAK_TOPS}}
        print("[bench] gather blend done", file=sys.stderr, flush=True)
    if not args.no_configs:
        out["colour_slices"] = run_colour_slices(adgi, torch)
        print("[bench] colour slices done", file=sys.stderr, flush=True)
    if not args.no_quality:
        out["quality"] = run_quality(adgi, torch, sc, cfg, tuning)
        print("[bench] quality done", file=sys.stderr, flush=True)
    chain_names = [c for c in args.chains.split(",") if c and c != "none"]
    if chain_names:
        out["chain_frames"] = {}
        for name in chain_names:
            c = CHAIN_CONFIGS[name]
            out["chain_frames"][name] = run_chains(
                adgi, torch, sc, storage if args.storage != "packed" else adgi.ADGI_FP32, tuning,
                args.steps, args.warmup, min(args.latency_frames, 20), c["chains"], c["steps"],
                c["burn_in"], c.get("dyn_chains", 0), c.get("dyn_steps", 0), c.get("dyn_burn_in", 0))
            print(f"[bench] chains {name} done", file=sys.stderr, flush=True)
    if not args.no_serve:
        out["serving"] = run_serving_child(args.serve_seconds)
        if "error" in out["serving"]:
            errors.append("serving: " + out["serving"]["error"])
        print(f"[bench] serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sc, cfg["budget"], cfg["n_min"], cfg["n_max"])
    out["errors"] = errors
    if errors:
        print("[bench] ERRORS: " + "; ".join(errors), file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
