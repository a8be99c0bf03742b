"""Lockstep parity driver: GPU library vs. FP64 CPU oracle, frame by frame.

Each frame the GPU runs ``adgi_update_probes`` with per-ray debug arrays on;
the oracle then runs the same frame on the same seeded inputs. Where FP32 and
FP64 can legitimately take different discrete decisions (a hit at a triangle
edge, a shadow ray grazing an occluder, a direction on a texel edge, a value on
a 10-bit code boundary), the oracle flags a tie and adopts the GPU's decision,
so both sides keep the same state; every other discrete disagreement counts
as a mismatch. Integer results (codes, scores, rays per probe, counts) must
then agree exactly and texels within the FP32 tolerance.
"""
from __future__ import annotations

import numpy as np

import oracle
import paper_2301_05125_amd as adgi


def rel_err(g: np.ndarray, o: np.ndarray, per_probe_axis: int = 0) -> np.ndarray:
    """|g-o| / max(|o|, 1e-3 * max over the probe's texels of |o|, 1e-8)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    flat = np.abs(o).reshape(o.shape[0], -1)
    floor = 1e-3 * flat.max(axis=1)
    floor = floor.reshape((-1,) + (1,) * (o.ndim - 1))
    den = np.maximum(np.maximum(np.abs(o), floor), 1e-8)
    return np.abs(g - o) / den


def f16_quantum(o) -> np.ndarray:
    """Spacing of binary16 values at |o|: 2^-24 below 2^-14 (subnormals),
    else 2^(floor(log2 |o|) - 10)."""
    a = np.abs(np.asarray(o, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
    return np.where(a < 2.0 ** -14, 2.0 ** -24, 2.0 ** (e - 10))


def texel_error_report(gi, gd, oi, od) -> dict:
    """Per-texel relative error distribution (same floor as the parity bar)."""
    out = {}
    for name, g, o in (("irradiance", gi, oi), ("depth", gd, od)):
        e = rel_err(g, o).ravel()
        out[name] = {"texels": int(e.size), "max": float(e.max(initial=0.0)),
                     "p99": float(np.percentile(e, 99)) if e.size else 0.0,
                     "p50": float(np.percentile(e, 50)) if e.size else 0.0,
                     "mean": float(e.mean()) if e.size else 0.0}
    return out


# Per-ray radiance bar. The GPU shades at an FP32 hit point and the oracle
# at an FP64 one. Origin and direction carry a few FP32 ulps, ~1e-6
# (|p|_inf + t) across the ray; where the ray meets the triangle at a
# glancing angle (|n.d| small) that offset slides the hit point along the
# surface by 1/|n.d| times as much, so dx = 1e-6 (|p|_inf + t) / |n.d|. The
# FP32 normal differs by an angle of about RAY_NORMAL_EPS. The direct light of light l,
# I_l cos(theta_l)/|l|^2, then moves by a relative
#   tan(theta_l) (dx/|l| + eps_n) + 2 dx/|l|
# (d ln cos / dx = tan(theta)/|l|, d ln |l|^-2 / dx = 2/|l|), which only
# grows large when the light grazes the surface (theta -> 90 degrees). The
# bar of a ray is RAY_RGB_BASE plus that term weighted by each light's share
# of the channel's radiance, the worst channel taken.
RAY_RGB_BASE = 1e-5
RAY_DX_REL = 1e-6
RAY_NORMAL_EPS = 1e-6


# Hit distance bar: 1e-5 relative plus the same glancing-angle slide of the
# hit point, dt = 1e-6 (|p|_inf + t) / |n.d|.
RAY_T_BASE = 1e-5


def probe_positions(scene, sel) -> np.ndarray:
    dims = scene.grid_dims.astype(np.int64)
    org = scene.grid_origin.astype(np.float64)
    spc = scene.grid_spacing.astype(np.float64)
    sel = np.asarray(sel, np.int64)
    pidx = np.stack([sel % dims[0], (sel // dims[0]) % dims[1], sel // (dims[0] * dims[1])], axis=1)
    return org + pidx * spc


def ray_t_bar(scene, frame, p, d, t, tri) -> np.ndarray:
    """Relative hit-distance bar of rays from p along unit d that hit
    triangle tri at distance t (misses: the base bar)."""
    bar = np.full(t.shape[0], RAY_T_BASE)
    hit = (tri >= 0) & np.isfinite(t) & (t > 0)
    if not hit.any():
        return bar
    V = scene.positions_at(frame).astype(np.float64)
    T = scene.indices[tri[hit]]
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    cos_in = np.maximum(np.abs(np.einsum("ij,ij->i", nrm, d[hit])), 1e-3)
    bar[hit] += RAY_DX_REL * (np.abs(p[hit]).max(axis=1) + t[hit]) / (cos_in * t[hit])
    return bar


def ray_rgb_bar(scene, frame, sel, n_sel, R, o, tri, shadow) -> np.ndarray:
    """Relative radiance bar of every traced ray of the tracked probes (the
    oracle's ray order: probe by probe, rays in index order)."""
    total = int(np.sum(n_sel))
    bar = np.full(total, RAY_RGB_BASE)
    if total == 0 or scene.num_lights == 0:
        return bar
    dims = scene.grid_dims.astype(np.int64)
    org = scene.grid_origin.astype(np.float64)
    spc = scene.grid_spacing.astype(np.float64)
    sel = np.asarray(sel, np.int64)
    pidx = np.stack([sel % dims[0], (sel // dims[0]) % dims[1], sel // (dims[0] * dims[1])], axis=1)
    pos_p = org + pidx * spc
    d = np.concatenate([oracle.probe_ray_dirs(int(k), R) if k else np.zeros((0, 3)) for k in n_sel])
    p = np.repeat(pos_p, np.asarray(n_sel, np.int64), axis=0)
    t = o[:, 3]
    lit = (tri >= 0) & np.isfinite(t) & (np.abs(o[:, :3]).max(axis=1) > 0)
    if not lit.any():
        return bar
    V = scene.positions_at(frame).astype(np.float64)
    T = scene.indices[tri[lit]]
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    dl = d[lit]
    nrm *= -np.sign(np.einsum("ij,ij->i", nrm, dl))[:, None]  # the side the ray came from
    x = p[lit] + t[lit, None] * dl
    cos_in = np.maximum(np.abs(np.einsum("ij,ij->i", nrm, dl)), 1e-3)
    dx = RAY_DX_REL * (np.abs(p[lit]).max(axis=1) + t[lit]) / cos_in
    lp = scene.light_positions(frame).astype(np.float64)
    li = scene.light_intensity.astype(np.float64)
    num = np.zeros((x.shape[0], 3))
    den = np.zeros((x.shape[0], 3))
    for l in range(lp.shape[0]):
        ell = lp[l] - x
        dist = np.linalg.norm(ell, axis=1)
        cos = np.einsum("ij,ij->i", nrm, ell) / dist
        vis = ((shadow[lit] >> l) & 1).astype(bool) & (cos > 0)
        cosc = np.where(vis, cos, 1.0)
        tan = np.sqrt(np.maximum(0.0, 1.0 - cosc * cosc)) / cosc
        sens = tan * (dx / dist + RAY_NORMAL_EPS) + 2.0 * dx / dist
        w = np.where(vis, cos / (dist * dist), 0.0)[:, None] * li[l][None, :]
        num += w * sens[:, None]
        den += w
    term = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0).max(axis=1)
    bar[lit] += term
    return bar


def gpu_scene_update(vol, scene, frame):
    if scene.anim_vertices and frame > 0:
        vol.update_scene(scene.positions_at(frame), light_pos=scene.light_positions(frame),
                         light_intensity=scene.light_intensity, sky=scene.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, scene.anim_vertices))
    else:
        vol.update_scene(scene.positions, light_pos=scene.light_positions(frame),
                         light_intensity=scene.light_intensity, sky=scene.sky,
                         mode=adgi.ADGI_SCENE_REFIT, refit_range=(0, 0))


def run_lockstep(scene, frames: int, adaptive: bool, n_uniform: int = 64, budget: int = 0,
                 n_min: int = 8, n_max: int = 2048, probes=None, storage=adgi.ADGI_FP32,
                 seed: int = 0x5EED, max_rays=None, tuning=None, check_rays: bool = True,
                 use_bvh: bool = True, fp64_twin: bool = False, gather: bool = False,
                 pilot_reuse: bool = False) -> dict:
    """``fp64_twin`` also runs an oracle that keeps its texels in FP64 (no
    binary16 rounding at the frame store), fed the same tie decisions, and
    returns per-texel error distributions against it."""
    P = scene.num_probes
    if max_rays is None:
        max_rays = max(budget, P * n_uniform, 1)
    vol = adgi.volume_for_scene(scene, storage=storage, max_rays=max_rays, seed=seed, debug=True,
                                blend_mode=adgi.ADGI_BLEND_GATHER if gather else adgi.ADGI_BLEND_SAMPLE)
    if tuning:
        vol.set_tuning(**tuning)
    fp16 = storage == adgi.ADGI_FP16
    packed = storage == adgi.ADGI_PACKED
    ora = oracle.OracleVolume(scene, seed=seed, fp16=fp16, probes=probes, use_bvh=use_bvh, gather=gather)
    sel = ora.probes
    ri, rd = vol.desc.irr_res - 2, vol.desc.depth_res - 2
    if packed:
        # the packed words follow from the GPU's samples through the oracle's
        # FP32 word update (the codes are FP32 decisions by the paper's precision)
        pk_irr = np.zeros((len(sel), ri * ri), np.uint32)
        pk_dep = np.zeros((len(sel), rd * rd), np.uint32)
        spacing = np.asarray(vol.desc.spacing[:], np.float64)
        s_diag = np.float32(np.sqrt(np.sum(spacing * spacing)))
        pk_inv_s = float(np.float32(1.0) / s_diag)
        pk_alpha = oracle.packed_alpha_table(vol.desc.hysteresis)
        res_pk = {"packed_word_mismatch": 0, "packed_border_mismatch": 0}
    twin = (oracle.OracleVolume(scene, seed=seed, fp16=False, probes=probes, use_bvh=use_bvh)
            if fp64_twin else None)
    res = {"mismatches": 0, "max_rel_irr": 0.0, "max_rel_depth": 0.0, "max_rel_ray": 0.0,
           "ties": {}, "frames": frames, "rays": 0, "count_mismatch": 0, "score_mismatch": 0,
           "alloc_mismatch": 0, "rotation_mismatch": 0, "max_rel_t": 0.0, "code_mismatch": 0,
           "pilot_rays": 0, "ray_bar_excess": 0, "rays_above_1e5": 0, "max_ray_over_bar": 0.0}
    for f in range(frames):
        if f > 0:
            gpu_scene_update(vol, scene, f)
        st = vol.update_probes(f, adaptive=adaptive, budget=budget, n_min=n_min, n_max=n_max,
                               n_uniform=n_uniform, sync=True, pilot_reuse=pilot_reuse)
        rb = vol.read_probes(texels=True, debug=True)
        R = oracle.frame_rotation(seed, f).reshape(9)
        if not np.array_equal(R, rb["frame_rotation"]):
            res["rotation_mismatch"] += 1
        hints = {"hit_tri": rb["hit_tri"], "shadow_bits": rb["shadow_bits"],
                 "irr_bin": rb["irr_bin"], "depth_bin": rb["depth_bin"],
                 "qv": rb["q10_vis"], "qr": rb["q10_rad"],
                 "pilot_tri": rb["pilot_tri"], "pilot_shadow": rb["pilot_shadow"]}
        if pilot_reuse and f % 2 == 0:
            hints.update(pilot_ibin=rb["pilot_ibin"], pilot_dbin=rb["pilot_dbin"])
        if gather:  # the gather blend takes every texel; no bin decisions
            del hints["irr_bin"], hints["depth_bin"]
        out = ora.update(f, adaptive=adaptive, budget=budget, n_min=n_min, n_max=n_max,
                         n_uniform=n_uniform, hints=hints, keep_rays=check_rays, pilot_reuse=pilot_reuse)
        if twin is not None:
            twin.update(f, adaptive=adaptive, budget=budget, n_min=n_min, n_max=n_max,
                        n_uniform=n_uniform, hints=hints, pilot_reuse=pilot_reuse)
        if adaptive and pilot_reuse and f % 2 == 0:
            # the reused pilot records: hit distance and radiance per pilot
            # (the oracle adopted the GPU's pilot hit decisions at ties; any
            # other disagreement is a counted hit mismatch)
            # (tracked probes' pilots)
            ridx = (8 * np.asarray(sel, np.int64)[:, None] + np.arange(8)[None, :]).reshape(-1)
            pr = rb["pilot_record"].astype(np.float64)[ridx]
            ot, gt = out["pilot_t"][ridx], pr[:, 3]
            miss = np.isinf(ot) | np.isinf(gt)
            res["pilot_miss_mismatch"] = res.get("pilot_miss_mismatch", 0) + \
                int(np.count_nonzero(np.isinf(ot) != np.isinf(gt)))
            et = np.abs(np.where(miss, 0.0, gt) - np.where(miss, 0.0, ot)) / np.maximum(np.abs(np.where(miss, 1.0, ot)), 1e-8)
            res["max_rel_pilot_t"] = max(res.get("max_rel_pilot_t", 0.0), float(et.max(initial=0.0)))
            pp = np.repeat(probe_positions(scene, sel), 8, axis=0)
            pd = np.array([oracle.pilot_dir(seed, int(r) // 8, int(r) % 8, f // 2) for r in ridx])
            tbar = ray_t_bar(scene, f, pp, pd, ot, rb["pilot_tri"][ridx])
            res["pilot_t_bar_excess"] = res.get("pilot_t_bar_excess", 0) + int(np.count_nonzero(et > tbar))
            eg = np.abs(pr[:, :3] - out["pilot_rgb"][ridx]).max(axis=1) / \
                np.maximum(np.abs(out["pilot_rgb"][ridx]).max(axis=1), 1e-6)
            res["max_rel_pilot_rgb"] = max(res.get("max_rel_pilot_rgb", 0.0), float(eg.max(initial=0.0)))
            res["pilot_samples"] = res.get("pilot_samples", 0) + int(len(sel) * 8)
        c = out["counts"]
        mism = c["hit_mismatch"] + c["shadow_mismatch"] + c["bin_mismatch"] + c["q10_mismatch"]
        if adaptive:
            res["score_mismatch"] += int(np.count_nonzero(out["score"] != rb["score"]))
            # the pilot codes of every probe and octant, this frame (even frames
            # too, and probes whose trigger sums are zero): after the oracle has
            # adopted the GPU's code at its flagged ties they must be identical
            res["code_mismatch"] += int(np.count_nonzero(out["qv"] != rb["q10_vis"])) + \
                int(np.count_nonzero(out["qr"] != rb["q10_rad"]))
            res["pilot_rays"] += int(out["qv"].size)
        res["alloc_mismatch"] += int(np.count_nonzero(out["n"] != rb["rays_per_probe"]))
        res["mismatches"] += mism
        for k in ("hit_ties", "shadow_ties", "bin_ties", "q10_ties"):
            res["ties"][k] = res["ties"].get(k, 0) + c[k]
        res["rays"] += c["rays"]
        res["stats_last"] = st
        # texels of the tracked probes
        gi = rb["irradiance"][sel]
        gd = rb["depth"][sel]
        oi = ora.irradiance_tiles()
        od = ora.depth_tiles()
        if packed:
            oracle.packed_blend(rb["rays_per_probe"][sel], rb["ray_offsets"][sel], rb["ray_record"],
                                rb["irr_bin"], rb["depth_bin"], ri, rd, pk_inv_s,
                                float(np.float32(vol.desc.tau_max)), pk_alpha, pk_irr, pk_dep)
            wi, wd = rb["irr_words"][sel], rb["depth_words"][sel]
            res_pk["packed_word_mismatch"] += int(np.count_nonzero(
                wi[:, 1:-1, 1:-1].reshape(len(sel), -1) != pk_irr)) + int(np.count_nonzero(
                    wd[:, 1:-1, 1:-1].reshape(len(sel), -1) != pk_dep))
            for q in range(len(sel)):
                fi = oracle.fold_tile(pk_irr[q].astype(np.float64), ri, 1).reshape(ri + 2, ri + 2)
                fd = oracle.fold_tile(pk_dep[q].astype(np.float64), rd, 1).reshape(rd + 2, rd + 2)
                res_pk["packed_border_mismatch"] += int(np.count_nonzero(fi != wi[q])) + \
                    int(np.count_nonzero(fd != wd[q]))
        ei, ed = rel_err(gi, oi), rel_err(gd, od)
        if fp16:
            # Both sides round to binary16 at the frame store, the GPU from FP32 and
            # the oracle from FP64: a value within rounding distance of a binary16
            # midpoint may land one quantum apart (a rounding tie). One quantum is
            # below the relative bar for normal halves, above it only for subnormal
            # ones, so such texels are counted here and excluded from the maximum.
            qi = np.abs(gi.astype(np.float64) - oi) <= f16_quantum(oi)
            qd = np.abs(gd.astype(np.float64) - od) <= f16_quantum(od)
            res["f16_quantum_ties"] = res.get("f16_quantum_ties", 0) + \
                int(np.count_nonzero(qi & (ei > 0))) + int(np.count_nonzero(qd & (ed > 0)))
            ei, ed = np.where(qi, 0.0, ei), np.where(qd, 0.0, ed)
        res["max_rel_irr"] = max(res["max_rel_irr"], float(ei.max(initial=0.0)))
        res["max_rel_depth"] = max(res["max_rel_depth"], float(ed.max(initial=0.0)))
        cnt_i = rb["irr_count"][sel].reshape(len(sel), -1)
        cnt_d = rb["depth_count"][sel].reshape(len(sel), -1)
        cap = 63 if packed else 255
        res["count_mismatch"] += int(np.count_nonzero(cnt_i != np.minimum(ora.irr_n, cap))) + \
            int(np.count_nonzero(cnt_d != np.minimum(ora.dep_n, cap)))
        if check_rays:
            base = rb["ray_offsets"][sel]
            n_sel = out["n"][sel]
            idx = np.concatenate([np.arange(b, b + k) for b, k in zip(base, n_sel)])
            owner = np.repeat(np.arange(len(sel)), n_sel)
            g = rb["ray_record"][idx].astype(np.float64)
            o = out["rays"]
            same = rb["hit_tri"][idx] == out["tri"]
            miss_g, miss_o = np.isinf(g[:, 3]), np.isinf(o[:, 3])
            res["mismatches"] += int(np.count_nonzero(miss_g != miss_o))
            gt = np.where(miss_g, 0.0, g[:, 3])
            ot = np.where(miss_o, 0.0, o[:, 3])
            # per-probe floor as for texels: 1e-3 x the probe's largest value
            peak_rgb = np.zeros(len(sel))
            np.maximum.at(peak_rgb, owner, np.abs(o[:, :3]).max(axis=1))
            peak_t = np.zeros(len(sel))
            np.maximum.at(peak_t, owner, np.abs(ot))
            den_rgb = np.maximum(np.maximum(np.abs(o[:, :3]), 1e-3 * peak_rgb[owner][:, None]), 1e-8)
            den_t = np.maximum(np.maximum(np.abs(ot), 1e-3 * peak_t[owner]), 1e-8)
            e = (np.abs(g[:, :3] - o[:, :3]) / den_rgb).max(axis=1)
            e = np.where(same, e, 0.0)
            bar = ray_rgb_bar(scene, f, sel, n_sel, out["R"], o, out["tri"], out["shadow"])
            res["rays_above_1e5"] += int(np.count_nonzero(e > RAY_RGB_BASE))
            res["ray_bar_excess"] += int(np.count_nonzero(e > bar))
            if e.size:
                res["max_ray_over_bar"] = max(res["max_ray_over_bar"], float((e / bar).max()))
            et = np.where(same, np.abs(gt - ot) / den_t, 0.0)
            res["max_rel_t"] = max(res.get("max_rel_t", 0.0), float(et.max(initial=0.0)))
            pr = np.repeat(probe_positions(scene, sel), np.asarray(n_sel, np.int64), axis=0)
            dr = np.concatenate([oracle.probe_ray_dirs(int(k), out["R"]) if k else np.zeros((0, 3)) for k in n_sel])
            tbar = ray_t_bar(scene, f, pr, dr, np.where(miss_o, np.inf, o[:, 3]), out["tri"])
            res["t_bar_excess"] = res.get("t_bar_excess", 0) + int(np.count_nonzero(et > tbar))
            k = int(np.argmax(e)) if e.size else 0
            if e.size and e[k] > res["max_rel_ray"]:
                res["max_rel_ray"] = float(e[k])
                res["worst_ray"] = {"gpu": g[k].tolist(), "oracle": o[k].tolist(),
                                    "tri": int(out["tri"][k]), "frame": f, "bar": float(bar[k])}
            k = int(np.argmax(e / bar)) if e.size else 0
            if e.size and e[k] / bar[k] >= res["max_ray_over_bar"]:
                res["worst_ray_vs_bar"] = {"gpu": g[k].tolist(), "oracle": o[k].tolist(), "err": float(e[k]),
                                           "tri": int(out["tri"][k]), "frame": f, "bar": float(bar[k]),
                                           "probe": int(sel[owner[k]])}
    if packed:
        res.update(res_pk)
    res["vs_oracle"] = texel_error_report(rb["irradiance"][sel], rb["depth"][sel],
                                          ora.irradiance_tiles(), ora.depth_tiles())
    res["mean_count"] = {"irradiance": float(ora.irr_n.mean()), "depth": float(ora.dep_n.mean())}
    if twin is not None:
        res["vs_fp64"] = texel_error_report(rb["irradiance"][sel], rb["depth"][sel],
                                            twin.irradiance_tiles(), twin.depth_tiles())
        res["oracle_vs_fp64"] = texel_error_report(ora.irradiance_tiles(), ora.depth_tiles(),
                                                   twin.irradiance_tiles(), twin.depth_tiles())
    res["irr_gpu"] = rb["irradiance"][sel]
    res["irr_oracle"] = ora.irradiance_tiles()
    res["oracle_counts"] = ora.counts.as_dict()
    vol.destroy_volume()
    return res


def scene_res(vol):
    return vol.desc.irr_res - 2, vol.desc.depth_res - 2


def run_chain_lockstep(scene, frames: int, chains: int, steps: int, burn_in: int,
                       sigma_pos: float = 0.5, warm_uniform: int = 2, n_uniform: int = 64,
                       storage=adgi.ADGI_FP32, seed: int = 0x5EED, tuning=None, dyn_chains: int = 0,
                       dyn_steps: int = 16, dyn_burn_in: int = 3, dyn_hysteresis: float = 0.91,
                       max_rays=None, pilot_reuse: bool = False) -> dict:
    """Chain frames (ADGI_MODE_CHAIN) in lockstep with the oracle's static
    Metropolis sampler, after ``warm_uniform`` uniform frames that give the
    guide a previous irradiance. Every probe is tracked (the guide reads any
    probe's texels). Each frame the oracle starts from the chain state the GPU
    left (FP32 values, so FP32/FP64 step rounding does not accumulate across
    frames), adopts the GPU's accept decisions only where it flags a tie, and
    must then produce the same samples: probes exactly, uv within 1e-4.
    With dyn_chains, the dynamic chains run too: the same for their state,
    accept decisions and marks, F exactly (FP32 of the same integers), and
    the per-probe dynamic ray counts exactly."""
    P = scene.num_probes
    samples = chains * (steps - burn_in - 1)
    if max_rays is None:
        max_rays = max(2 * samples + (P * 232 if dyn_chains else 0), P * n_uniform)
    vol = adgi.volume_for_scene(scene, storage=storage, max_rays=max_rays, seed=seed, debug=True,
                                max_chains=max(chains, dyn_chains))
    if tuning:
        vol.set_tuning(**tuning)
    fp16 = storage == adgi.ADGI_FP16
    ora = oracle.OracleVolume(scene, seed=seed, fp16=fp16)
    cp = oracle.ChainParams(chains, steps, burn_in, float(np.float32(sigma_pos)),
                            float(np.float32(adgi.CHAIN_SIGMA_DIR)))
    state = np.zeros((chains, 5), np.float64)
    dp = None
    if dyn_chains:
        dp = oracle.ChainParams(dyn_chains, dyn_steps, dyn_burn_in, float(np.float32(1.5)),
                                float(np.float32(6 * adgi.CHAIN_SIGMA_DIR)))
    dstate = np.zeros((max(dyn_chains, 1), 5), np.float64)
    res = {"mark_mismatch": 0, "F_mismatch": 0, "dyn_ray_mismatch": 0, "dyn_accept_mismatch": 0,
           "marks": 0, "dyn_rays": 0, "max_dyn_state_err": 0.0,"mismatches": 0, "max_rel_irr": 0.0, "max_rel_depth": 0.0, "count_mismatch": 0,
           "alloc_mismatch": 0, "code_mismatch": 0, "accept_mismatch": 0, "probe_mismatch": 0,
           "sample_count_mismatch": 0, "max_uv_err": 0.0, "max_state_err": 0.0, "ties": {},
           "frames": frames, "samples": 0, "accept_rate": 0.0, "max_rel_ray": 0.0, "rays": 0,
           "pilot_rays": 0}
    for f in range(warm_uniform + frames):
        if f > 0:
            gpu_scene_update(vol, scene, f)
        chain = f >= warm_uniform
        if chain:
            st = vol.update_chains(f, chains, steps, burn_in, sigma_pos=sigma_pos, sync=True,
                                   dyn_chains=dyn_chains, dyn_steps=dyn_steps, dyn_burn_in=dyn_burn_in,
                                   dyn_hysteresis=dyn_hysteresis, pilot_reuse=pilot_reuse)
        else:
            st = vol.update_probes(f, adaptive=False, n_uniform=n_uniform, sync=True)
        rb = vol.read_probes(texels=True, debug=True)
        hints = {"hit_tri": rb["hit_tri"], "shadow_bits": rb["shadow_bits"],
                 "irr_bin": rb["irr_bin"], "depth_bin": rb["depth_bin"],
                 "qv": rb["q10_vis"], "qr": rb["q10_rad"]}
        if chain:
            hints.update(pilot_tri=rb["pilot_tri"], pilot_shadow=rb["pilot_shadow"])
            if pilot_reuse and f % 2 == 0:
                hints.update(pilot_ibin=rb["pilot_ibin"], pilot_dbin=rb["pilot_dbin"])
            hints["accept"] = rb["chain_accept"].reshape(-1)
            if dyn_chains:
                hints["dyn_accept"] = rb["dyn_accept"].reshape(-1)
            out = ora.chain_update(f, cp, state, init=(f == warm_uniform), hints=hints, dyn=dp,
                                   dyn_state=dstate[:dyn_chains] if dyn_chains else None,
                                   dyn_init=(f == warm_uniform), h_dyn=dyn_hysteresis,
                                   pilot_reuse=pilot_reuse)
            if dyn_chains:
                res["F_mismatch"] += int(np.count_nonzero(
                    out["F"].astype(np.float32) != rb["dyn_target"].reshape(-1)))
                res["mark_mismatch"] += int(np.count_nonzero(out["mark"] != rb["dyn_mark"].reshape(-1)))
                res["marks"] += int(out["mark"].sum())
                res["dyn_accept_mismatch"] += int(np.count_nonzero(out["dyn_accept"] != hints["dyn_accept"]))
                res["dyn_ray_mismatch"] += int(np.count_nonzero(out["dyn_offsets"] != rb["dyn_ray_offsets"]))
                res["dyn_rays"] += int(out["dyn_offsets"][-1])
                res["max_dyn_state_err"] = max(res["max_dyn_state_err"], float(np.abs(
                    rb["dyn_state"].astype(np.float64) - dstate[:dyn_chains]).max(initial=0.0)))
                dstate[:dyn_chains] = rb["dyn_state"].astype(np.float64)
            res["code_mismatch"] += int(np.count_nonzero(out["qv"] != rb["q10_vis"])) + \
                int(np.count_nonzero(out["qr"] != rb["q10_rad"]))
            res["pilot_rays"] += int(out["qv"].size)
            res["accept_mismatch"] += int(np.count_nonzero(out["accept"] != hints["accept"]))
            res["accept_rate"] = float(np.mean(out["accept"]))
            sp_o = out["sample_probe"][out["perm"]]
            suv_o = out["sample_uv"][out["perm"]]
            if rb["num_samples"] != len(sp_o) or \
                    st["primary_rays"] != 2 * len(sp_o) + (int(out["dyn_offsets"][-1]) if dyn_chains else 0):
                res["sample_count_mismatch"] += 1
            else:
                res["probe_mismatch"] += int(np.count_nonzero(rb["sample_probe"] != sp_o))
                res["max_uv_err"] = max(res["max_uv_err"], float(np.abs(
                    rb["sample_uv"].astype(np.float64) - suv_o).max(initial=0.0)))
            res["max_state_err"] = max(res["max_state_err"], float(np.abs(
                rb["chain_state"].astype(np.float64) - state).max(initial=0.0)))
            res["samples"] += len(sp_o)
            # the next frame starts where the GPU's chains stopped
            state[:] = rb["chain_state"].astype(np.float64)
            c = out["counts"]
            res["mismatches"] += c["chain_mismatch"] + c["q10_mismatch"]
            for k in ("chain_ties", "q10_ties"):
                res["ties"][k] = res["ties"].get(k, 0) + c[k]
        else:
            out = ora.update(f, adaptive=False, n_uniform=n_uniform, hints=hints)
            c = out["counts"]
        res["mismatches"] += c["hit_mismatch"] + c["shadow_mismatch"] + c["bin_mismatch"]
        for k in ("hit_ties", "shadow_ties", "bin_ties"):
            res["ties"][k] = res["ties"].get(k, 0) + c[k]
        res["rays"] += c["rays"]
        res["alloc_mismatch"] += int(np.count_nonzero(out["n"] != rb["rays_per_probe"]))
        ei = rel_err(rb["irradiance"], ora.irradiance_tiles())
        ed = rel_err(rb["depth"], ora.depth_tiles())
        if fp16:
            qi = np.abs(rb["irradiance"].astype(np.float64) - ora.irradiance_tiles()) <= \
                f16_quantum(ora.irradiance_tiles())
            qd = np.abs(rb["depth"].astype(np.float64) - ora.depth_tiles()) <= \
                f16_quantum(ora.depth_tiles())
            res["f16_quantum_ties"] = res.get("f16_quantum_ties", 0) + \
                int(np.count_nonzero(qi & (ei > 0))) + int(np.count_nonzero(qd & (ed > 0)))
            ei, ed = np.where(qi, 0.0, ei), np.where(qd, 0.0, ed)
        res["max_rel_irr"] = max(res["max_rel_irr"], float(ei.max(initial=0.0)))
        res["max_rel_depth"] = max(res["max_rel_depth"], float(ed.max(initial=0.0)))
        res["count_mismatch"] += int(np.count_nonzero(
            rb["irr_count"].reshape(P, -1) != np.minimum(ora.irr_n, 255))) + int(np.count_nonzero(
                rb["depth_count"].reshape(P, -1) != np.minimum(ora.dep_n, 255)))
        res["stats_last"] = st
    res["vs_oracle"] = texel_error_report(rb["irradiance"], rb["depth"], ora.irradiance_tiles(),
                                          ora.depth_tiles())
    res["oracle_counts"] = ora.counts.as_dict()
    vol.destroy_volume()
    return res
