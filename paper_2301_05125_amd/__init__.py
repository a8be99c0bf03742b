"""Python binding of the gfx950 probe-update library (ctypes, marshalling only).

Every step of the probe update runs in the HIP kernels of ``libadgi.so``;
this module only converts numpy arrays and Python values to the C ABI of
``include/adgi.h``. PyTorch provides device memory (its caching allocator, as
the library's allocator callbacks) and the caller's stream. The import fails
loudly when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadgi.so")

ADGI_OK = 0
STATUS = {0: "ADGI_OK", -1: "ADGI_ERR_INVALID_ARG", -2: "ADGI_ERR_OUT_OF_MEMORY",
          -3: "ADGI_ERR_BUDGET", -4: "ADGI_ERR_NO_SCENE", -5: "ADGI_ERR_TOPOLOGY",
          -6: "ADGI_ERR_DEVICE"}
(ADGI_ERR_INVALID_ARG, ADGI_ERR_OUT_OF_MEMORY, ADGI_ERR_BUDGET, ADGI_ERR_NO_SCENE,
 ADGI_ERR_TOPOLOGY, ADGI_ERR_DEVICE) = -1, -2, -3, -4, -5, -6
ADGI_FP32, ADGI_FP16, ADGI_PACKED = 0, 1, 2
ADGI_SCENE_REBUILD, ADGI_SCENE_REFIT = 0, 1
ADGI_DEBUG_ARRAYS = 1
ADGI_STATIC_SCRATCH = 2
ADGI_STATIC_SCRATCH_BYTES = 64 << 20
ADGI_MODE_UNIFORM, ADGI_MODE_ADAPTIVE, ADGI_MODE_CHAIN = 0, 1, 2
ADGI_BLEND_SAMPLE, ADGI_BLEND_GATHER = 0, 1
CHAIN_MAX_STEPS = 256
CHAIN_SIGMA_DIR = math.sqrt(math.pi / 256.0)  # default octahedral step of the chains (Sec. 4.8)
MAX_LIGHTS = 8
TAU_MAX = (math.exp(5.0) - 1.0) / 15.0


class AdgiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class VolumeDesc(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("spacing", C.c_float * 3), ("dims", C.c_int32 * 3),
                ("irr_res", C.c_int32), ("depth_res", C.c_int32), ("storage", C.c_int32),
                ("hysteresis", C.c_float), ("tau_max", C.c_float),
                ("max_rays_per_frame", C.c_int64), ("seed", C.c_uint64), ("flags", C.c_uint32),
                ("max_chains", C.c_int32), ("blend_mode", C.c_int32)]


class SceneDesc(C.Structure):
    _fields_ = [("positions", C.c_void_p), ("num_vertices", C.c_int32), ("indices", C.c_void_p),
                ("num_triangles", C.c_int32), ("albedo", C.c_void_p), ("light_pos", C.c_void_p),
                ("light_intensity", C.c_void_p), ("num_lights", C.c_int32), ("sky", C.c_float * 3),
                ("mode", C.c_int32), ("refit_vertex_begin", C.c_int32),
                ("refit_vertex_end", C.c_int32)]


class UpdateParams(C.Structure):
    _fields_ = [("frame", C.c_int32), ("adaptive", C.c_int32), ("budget", C.c_int64),
                ("n_min", C.c_int32), ("n_max", C.c_int32), ("n_uniform", C.c_int32),
                ("beta", C.c_float), ("mu", C.c_int32), ("theta", C.c_int32), ("sync", C.c_int32),
                ("chain_count", C.c_int32), ("chain_steps", C.c_int32), ("chain_burn_in", C.c_int32),
                ("chain_sigma_pos", C.c_float), ("chain_sigma_dir", C.c_float),
                ("chain_reset", C.c_int32), ("dyn_chain_count", C.c_int32),
                ("dyn_chain_steps", C.c_int32), ("dyn_chain_burn_in", C.c_int32),
                ("dyn_sigma_pos", C.c_float), ("dyn_sigma_dir", C.c_float),
                ("dyn_hysteresis", C.c_float), ("pilot_reuse", C.c_int32)]


class UpdateStats(C.Structure):
    _fields_ = [("primary_rays", C.c_int64), ("pilot_rays", C.c_int64), ("shadow_rays", C.c_int64),
                ("budget_used", C.c_int64), ("lambda_", C.c_uint32), ("n_min_seen", C.c_int32),
                ("n_max_seen", C.c_int32), ("ms_total", C.c_float), ("ms_stage", C.c_float * 8),
                ("ties", C.c_int64 * 4)]

    def as_dict(self):
        return {"primary_rays": self.primary_rays, "pilot_rays": self.pilot_rays,
                "shadow_rays": self.shadow_rays, "budget_used": self.budget_used,
                "lambda": self.lambda_, "n_min_seen": self.n_min_seen,
                "n_max_seen": self.n_max_seen, "ms_total": self.ms_total,
                "ms_stage": [float(x) for x in self.ms_stage[:8]]}


class ProbeReadback(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "irradiance", "depth", "irr_count", "depth_count", "rays_per_probe", "score",
        "ray_offsets", "hit_tri", "shadow_bits", "irr_bin", "depth_bin", "ray_record",
        "q10_vis", "q10_rad", "frame_rotation")] + [("num_rays", C.c_int64)] + \
        [("irr_words", C.c_void_p), ("depth_words", C.c_void_p)] + \
        [(n, C.c_void_p) for n in ("chain_state", "sample_probe", "sample_uv", "chain_accept")] + \
        [("num_samples", C.c_int64), ("num_chains", C.c_int32), ("chain_steps", C.c_int32)] + \
        [(n, C.c_void_p) for n in ("dyn_mark", "dyn_target", "dyn_state", "dyn_ray_offsets", "dyn_accept")] + \
        [("num_dyn_rays", C.c_int64), ("num_dyn_chains", C.c_int32), ("dyn_chain_steps", C.c_int32),
         ("proxy_dims", C.c_int32 * 3), ("reserved", C.c_int32)] + \
        [(n, C.c_void_p) for n in ("pilot_record", "pilot_tri", "pilot_shadow", "pilot_ibin", "pilot_dbin")]


class TraceWork(C.Structure):
    _fields_ = [("primary_rays", C.c_int64), ("shadow_rays", C.c_int64),
                ("node_tests", C.c_int64), ("tri_tests", C.c_int64), ("box_tests", C.c_int64),
                ("shade_node_tests", C.c_int64), ("shade_tri_tests", C.c_int64),
                ("shade_box_tests", C.c_int64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32),
                ("reserved", C.c_int32)]


class StreamDesc(C.Structure):
    _fields_ = [("volume", VolumeDesc), ("scene", SceneDesc), ("params", UpdateParams)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "admissions", "evictions",
                                         "primary_rays", "resident_bytes", "peak_resident_bytes")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "span_s",
                                          "admit_ms", "evict_ms", "device_busy_ms")]

    def as_dict(self):
        return {n: (float(getattr(self, n)) if t is C.c_double else int(getattr(self, n)))
                for n, t in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("persistent", C.c_int32), ("trace_block", C.c_int32),
                ("trace_waves_per_cu", C.c_int32), ("blend_chunk", C.c_int32),
                ("blend_blocks_per_cu", C.c_int32), ("bvh_width", C.c_int32),
                ("chain_lanes", C.c_int32), ("ray_order", C.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None
_live = weakref.WeakSet()


@atexit.register
def _destroy_live_volumes():
    """Release device state while torch (the allocator) is still alive."""
    for v in list(_live):
        v.destroy_volume()


def lib():
    """Load libadgi.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(no CPU fallback exists)")
        try:
            import torch  # (loads the HIP runtime torch uses)
            # the device is initialised through torch before the library
            # registers its kernels, as in every process it has run in
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.adgi_last_error.restype = C.c_char_p
        L.adgi_create_volume.argtypes = [P, P, P, P]
        L.adgi_update_scene.argtypes = [P, P]
        L.adgi_update_probes.argtypes = [P, P, P]
        L.adgi_update_probes_static.argtypes = [P, P, P]
        L.adgi_pack_channel.argtypes = [P, C.c_int64, C.c_int32, P, P, P]
        L.adgi_pack_channel.restype = C.c_int
        L.adgi_read_probes.argtypes = [P, P]
        L.adgi_destroy_volume.argtypes = [P]
        L.adgi_destroy_volume.restype = None
        L.adgi_get_tuning.argtypes = [P, P]
        L.adgi_set_tuning.argtypes = [P, P]
        L.adgi_autotune.argtypes = [P, P, P]
        L.adgi_measure_trace_work.argtypes = [P, P, P]
        L.adgi_state_size.argtypes = [P]
        L.adgi_state_size.restype = C.c_size_t
        L.adgi_save_state.argtypes = [P, P, C.c_size_t]
        L.adgi_restore_state.argtypes = [P, P, C.c_size_t]
        L.adgi_device_bytes.argtypes = [P]
        L.adgi_device_bytes.restype = C.c_size_t
        L.adgi_server_now_ns.restype = C.c_int64
        L.adgi_server_last_error.restype = C.c_char_p
        L.adgi_server_create.argtypes = [P, P, P]
        L.adgi_server_add_stream.argtypes = [P, P, P]
        L.adgi_server_set_budget.argtypes = [P, C.c_int64]
        L.adgi_server_stream_info.argtypes = [P, C.c_int32, P, P, P]
        L.adgi_server_submit.argtypes = [P, C.c_int32, P, C.c_int64]
        L.adgi_server_progress.argtypes = [P, P]
        L.adgi_server_drain.argtypes = [P]
        L.adgi_server_get_stats.argtypes = [P, P]
        L.adgi_server_latencies.argtypes = [P, P, C.c_int64, P]
        L.adgi_server_read_stream.argtypes = [P, C.c_int32, P]
        L.adgi_server_destroy.argtypes = [P]
        L.adgi_server_destroy.restype = None
        for name in ("adgi_server_create", "adgi_server_add_stream", "adgi_server_set_budget",
                     "adgi_server_stream_info", "adgi_server_submit", "adgi_server_progress",
                     "adgi_server_drain", "adgi_server_get_stats", "adgi_server_latencies",
                     "adgi_server_read_stream"):
            getattr(L, name).restype = C.c_int
        for name in ("adgi_create_volume", "adgi_update_scene", "adgi_update_probes", "adgi_update_probes_static",
                     "adgi_read_probes", "adgi_get_tuning", "adgi_set_tuning", "adgi_autotune",
                     "adgi_measure_trace_work",
                     "adgi_save_state", "adgi_restore_state"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != ADGI_OK:
        raise AdgiError(status, lib().adgi_last_error().decode())


def _check_server(status: int):
    if status != ADGI_OK:
        raise AdgiError(status, lib().adgi_server_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _torch_allocator():
    """Allocator callbacks backed by torch's caching allocator."""
    import torch
    dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream()

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
        except RuntimeError:
            return None

    def _free(ptr, ctx):
        if torch.cuda is not None:
            torch.cuda.caching_allocator_delete(int(ptr))

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return a


def create_volume(origin, spacing, dims, irr_res=8, depth_res=16, storage=ADGI_FP32,
                  hysteresis=0.97, tau_max=TAU_MAX, max_rays_per_frame=1 << 20, seed=1,
                  debug=False, stream=None, allocator="torch", max_chains=0,
                  blend_mode=ADGI_BLEND_SAMPLE, static_scratch=False) -> "Volume":
    return Volume(origin, spacing, dims, irr_res, depth_res, storage, hysteresis, tau_max,
                  max_rays_per_frame, seed, debug, stream, allocator, max_chains, blend_mode, static_scratch)


class Volume:
    """A probe volume: device state, scene and the per-frame update."""

    def __init__(self, origin, spacing, dims, irr_res=8, depth_res=16, storage=ADGI_FP32,
                 hysteresis=0.97, tau_max=TAU_MAX, max_rays_per_frame=1 << 20, seed=1,
                 debug=False, stream=None, allocator="torch", max_chains=0,
                 blend_mode=ADGI_BLEND_SAMPLE, static_scratch=False):
        d = VolumeDesc()
        d.origin[:] = [float(x) for x in origin]
        d.spacing[:] = [float(x) for x in spacing]
        d.dims[:] = [int(x) for x in dims]
        d.irr_res, d.depth_res, d.storage = int(irr_res), int(depth_res), int(storage)
        d.hysteresis, d.tau_max = float(hysteresis), float(tau_max)
        d.max_rays_per_frame = int(max_rays_per_frame)
        d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        d.flags = (ADGI_DEBUG_ARRAYS if debug else 0) | (ADGI_STATIC_SCRATCH if static_scratch else 0)
        d.max_chains = int(max_chains)
        d.blend_mode = int(blend_mode)
        self.desc = d
        self.P = int(np.prod([int(x) for x in dims]))
        self._alloc = None
        if allocator == "torch":
            import torch
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            self._alloc = _torch_allocator()
        elif allocator is not None:
            self._alloc = allocator
        self.stream = stream
        h = C.c_void_p()
        _check(lib().adgi_create_volume(C.byref(d), C.byref(self._alloc) if self._alloc else None,
                                        C.c_void_p(stream) if stream else None, C.byref(h)))
        self.h = h
        _live.add(self)

    def __del__(self):
        self.destroy_volume()

    def destroy_volume(self):
        if getattr(self, "h", None) and self.h.value:
            lib().adgi_destroy_volume(self.h)
            self.h = C.c_void_p()

    def update_scene(self, positions, indices=None, albedo=None, light_pos=None,
                     light_intensity=None, sky=(0.0, 0.0, 0.0), mode=ADGI_SCENE_REBUILD,
                     refit_range=None):
        pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
        idx = None if indices is None else np.ascontiguousarray(indices, np.int32).reshape(-1, 3)
        alb = None if albedo is None else np.ascontiguousarray(albedo, np.float32).reshape(-1, 3)
        lp = np.ascontiguousarray(light_pos if light_pos is not None else np.zeros((0, 3)),
                                  np.float32).reshape(-1, 3)
        li = np.ascontiguousarray(light_intensity if light_intensity is not None
                                  else np.zeros((0, 3)), np.float32).reshape(-1, 3)
        s = SceneDesc()
        s.positions = _ptr(pos)
        s.num_vertices = pos.shape[0]
        s.indices = _ptr(idx)
        s.num_triangles = 0 if idx is None else idx.shape[0]
        if mode == ADGI_SCENE_REFIT and idx is None:
            s.num_triangles = self._nt
        s.albedo = _ptr(alb)
        s.light_pos = _ptr(lp)
        s.light_intensity = _ptr(li)
        s.num_lights = lp.shape[0]
        s.sky[:] = [float(x) for x in sky]
        s.mode = int(mode)
        if refit_range is None:
            refit_range = (0, pos.shape[0])
        s.refit_vertex_begin, s.refit_vertex_end = int(refit_range[0]), int(refit_range[1])
        _check(lib().adgi_update_scene(self.h, C.byref(s)))
        if mode == ADGI_SCENE_REBUILD:
            self._nt = s.num_triangles

    def update_probes(self, frame, adaptive=False, budget=0, n_min=8, n_max=2048, n_uniform=64,
                      beta=5.0, mu=2, theta=8, sync=True, pilot_reuse=False) -> dict:
        p = UpdateParams(int(frame), 1 if adaptive else 0, int(budget), int(n_min), int(n_max),
                         int(n_uniform), float(beta), int(mu), int(theta), 1 if sync else 0)
        p.pilot_reuse = 1 if pilot_reuse else 0
        st = UpdateStats()
        _check(lib().adgi_update_probes(self.h, C.byref(p), C.byref(st)))
        return st.as_dict() if sync else {}

    def update_probes_static(self, frame, adaptive=False, budget=0, n_min=8, n_max=2048, n_uniform=64,
                             beta=5.0, mu=2, theta=8, sync=True, pilot_reuse=False) -> dict:
        """update_probes with the frame scratch in the library's fixed per-GPU
        array (no allocation, eager launches); budgeted and uniform frames."""
        p = UpdateParams(int(frame), 1 if adaptive else 0, int(budget), int(n_min), int(n_max),
                         int(n_uniform), float(beta), int(mu), int(theta), 1 if sync else 0)
        p.pilot_reuse = 1 if pilot_reuse else 0
        st = UpdateStats()
        _check(lib().adgi_update_probes_static(self.h, C.byref(p), C.byref(st)))
        return st.as_dict() if sync else {}

    @staticmethod
    def _chain_params(frame, chains, steps, burn_in, sigma_pos, sigma_dir, reset, beta, sync, mu=2, theta=8,
                      dyn_chains=0, dyn_steps=0, dyn_burn_in=0, dyn_sigma_pos=1.5,
                      dyn_sigma_dir=6 * CHAIN_SIGMA_DIR, dyn_hysteresis=0.91):
        return UpdateParams(int(frame), ADGI_MODE_CHAIN, 0, 1, 1, 1, float(beta), int(mu), int(theta),
                            1 if sync else 0, int(chains), int(steps), int(burn_in),
                            float(sigma_pos), float(sigma_dir), 1 if reset else 0, int(dyn_chains),
                            int(dyn_steps), int(dyn_burn_in), float(dyn_sigma_pos), float(dyn_sigma_dir),
                            float(dyn_hysteresis))

    def update_chains(self, frame, chains, steps, burn_in, sigma_pos=0.5, sigma_dir=CHAIN_SIGMA_DIR,
                      reset=False, beta=5.0, sync=True, mu=2, theta=8, dyn_chains=0, dyn_steps=0,
                      dyn_burn_in=0, dyn_sigma_pos=1.5, dyn_sigma_dir=6 * CHAIN_SIGMA_DIR,
                      dyn_hysteresis=0.91, pilot_reuse=False) -> dict:
        """One chain frame (ADGI_MODE_CHAIN): pilots and detection, `chains`
        static Metropolis chains of `steps` steps each (the first burn_in + 1
        emit nothing), two rays per sample; with dyn_chains > 0 also the
        dynamic chains on the 3x3x3 proxies and their texel-centre rays;
        blend."""
        p = self._chain_params(frame, chains, steps, burn_in, sigma_pos, sigma_dir, reset, beta, sync, mu,
                               theta, dyn_chains, dyn_steps, dyn_burn_in, dyn_sigma_pos, dyn_sigma_dir,
                               dyn_hysteresis)
        p.pilot_reuse = 1 if pilot_reuse else 0
        st = UpdateStats()
        _check(lib().adgi_update_probes(self.h, C.byref(p), C.byref(st)))
        return st.as_dict() if sync else {}

    def read_probes(self, texels=True, debug=False, probes=None) -> dict:
        d = self.desc
        P = self.P
        gi, gd = d.irr_res, d.depth_res
        out = {}
        rb = ProbeReadback()
        if texels:
            out["irradiance"] = np.zeros((P, gi, gi, 3), np.float32)
            out["depth"] = np.zeros((P, gd, gd, 2), np.float32)
            out["irr_count"] = np.zeros((P, gi - 2, gi - 2), np.uint8)
            out["depth_count"] = np.zeros((P, gd - 2, gd - 2), np.uint8)
        out["rays_per_probe"] = np.zeros(P, np.int32)
        out["score"] = np.zeros(P, np.int64)
        out["ray_offsets"] = np.zeros(P + 1, np.int64)
        out["q10_vis"] = np.zeros(P * 8, np.uint16)
        out["q10_rad"] = np.zeros(P * 8, np.uint16)
        out["frame_rotation"] = np.zeros(9, np.float32)
        if d.storage == ADGI_PACKED:
            out["irr_words"] = np.zeros((P, gi, gi), np.uint32)
            out["depth_words"] = np.zeros((P, gd, gd), np.uint32)
        for k, a in out.items():
            setattr(rb, k, _ptr(a))
        _check(lib().adgi_read_probes(self.h, C.byref(rb)))
        if d.max_chains > 0 and rb.num_chains > 0:
            Cn, M, S = int(rb.num_chains), int(rb.chain_steps), int(rb.num_samples)
            ch = {"chain_state": np.zeros((Cn, 5), np.float32),
                  "sample_probe": np.zeros(max(S, 1), np.uint32),
                  "sample_uv": np.zeros((max(S, 1), 2), np.float32)}
            if debug:
                ch["chain_accept"] = np.zeros((Cn, M), np.uint8)
            rb3 = ProbeReadback()
            for k, a in ch.items():
                setattr(rb3, k, _ptr(a))
            _check(lib().adgi_read_probes(self.h, C.byref(rb3)))
            ch["sample_probe"], ch["sample_uv"] = ch["sample_probe"][:S], ch["sample_uv"][:S]
            out.update(ch)
            out["num_samples"] = S
        if d.max_chains > 0:
            pdims = tuple(int(x) for x in rb.proxy_dims)
            Pp = pdims[0] * pdims[1] * pdims[2]
            Cd, Md = int(rb.num_dyn_chains), int(rb.dyn_chain_steps)
            dy = {"dyn_mark": np.zeros((Pp, 8), np.uint8), "dyn_target": np.zeros((Pp, 8), np.float32),
                  "dyn_ray_offsets": np.zeros(P + 1, np.int64)}
            if Cd:
                dy["dyn_state"] = np.zeros((Cd, 5), np.float32)
                if debug:
                    dy["dyn_accept"] = np.zeros((Cd, Md), np.uint8)
            rb4 = ProbeReadback()
            for k, a in dy.items():
                setattr(rb4, k, _ptr(a))
            _check(lib().adgi_read_probes(self.h, C.byref(rb4)))
            out.update(dy)
            out["proxy_dims"] = pdims
            out["num_dyn_rays"] = int(rb.num_dyn_rays)
        if debug:
            R = int(rb.num_rays)
            dbg = {"hit_tri": np.zeros(max(R, 1), np.int32),
                   "shadow_bits": np.zeros(max(R, 1), np.uint8),
                   "irr_bin": np.zeros(max(R, 1), np.uint16),
                   "depth_bin": np.zeros(max(R, 1), np.uint16),
                   "ray_record": np.zeros((max(R, 1), 4), np.float32),
                   "pilot_record": np.zeros((P * 8, 4), np.float32),
                   "pilot_tri": np.zeros(P * 8, np.int32),
                   "pilot_shadow": np.zeros(P * 8, np.uint8),
                   "pilot_ibin": np.zeros(P * 8, np.uint16),
                   "pilot_dbin": np.zeros(P * 8, np.uint16)}
            rb2 = ProbeReadback()
            for k, a in dbg.items():
                setattr(rb2, k, _ptr(a))
            _check(lib().adgi_read_probes(self.h, C.byref(rb2)))
            for k, a in dbg.items():
                out[k] = a if k.startswith("pilot_") else a[:R]
        out["num_rays"] = int(rb.num_rays)
        return out

    def query_irradiance(self, points, normals):
        """Irradiance [K][3] at points [K][3] with unit normals [K][3]
        (torch CUDA float32 tensors, or anything torch.as_tensor takes)."""
        import torch
        pts = torch.as_tensor(points, dtype=torch.float32, device="cuda").reshape(-1, 3).contiguous()
        nrm = torch.as_tensor(normals, dtype=torch.float32, device="cuda").reshape(-1, 3).contiguous()
        out = torch.empty_like(pts)
        _check(lib().adgi_query_irradiance(self.h, C.c_void_p(pts.data_ptr()), C.c_void_p(nrm.data_ptr()),
                                           C.c_int64(pts.shape[0]), C.c_void_p(out.data_ptr())))
        torch.cuda.current_stream().synchronize()
        return out

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().adgi_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        _check(lib().adgi_get_tuning(self.h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(lib().adgi_set_tuning(self.h, C.byref(t)))

    def autotune(self, frame, adaptive=False, budget=0, n_min=8, n_max=2048, n_uniform=64,
                 beta=5.0, mu=2, theta=8) -> dict:
        p = UpdateParams(int(frame), 1 if adaptive else 0, int(budget), int(n_min), int(n_max),
                         int(n_uniform), float(beta), int(mu), int(theta), 1)
        t = Tuning()
        _check(lib().adgi_autotune(self.h, C.byref(p), C.byref(t)))
        return t.as_dict()

    def measure_trace_work(self, frame, adaptive=False, budget=0, n_min=8, n_max=2048,
                           n_uniform=64, beta=5.0, mu=2, theta=8) -> dict:
        p = UpdateParams(int(frame), 1 if adaptive else 0, int(budget), int(n_min), int(n_max),
                         int(n_uniform), float(beta), int(mu), int(theta), 1)
        w = TraceWork()
        _check(lib().adgi_measure_trace_work(self.h, C.byref(p), C.byref(w)))
        return w.as_dict()

    def measure_chain_trace_work(self, frame, chains, steps, burn_in, sigma_pos=0.5,
                                 sigma_dir=CHAIN_SIGMA_DIR, beta=5.0, dyn_chains=0, dyn_steps=0,
                                 dyn_burn_in=0) -> dict:
        """Traversal work of a chain frame's rays (state restored after)."""
        p = self._chain_params(frame, chains, steps, burn_in, sigma_pos, sigma_dir, False, beta, True,
                               dyn_chains=dyn_chains, dyn_steps=dyn_steps, dyn_burn_in=dyn_burn_in)
        w = TraceWork()
        _check(lib().adgi_measure_trace_work(self.h, C.byref(p), C.byref(w)))
        return w.as_dict()

    def state_size(self) -> int:
        return int(lib().adgi_state_size(self.h))

    def save_state(self) -> np.ndarray:
        buf = np.zeros(self.state_size(), np.uint8)
        _check(lib().adgi_save_state(self.h, _ptr(buf), buf.nbytes))
        return buf

    def restore_state(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(lib().adgi_restore_state(self.h, _ptr(buf), buf.nbytes))

    def device_bytes(self) -> int:
        return int(lib().adgi_device_bytes(self.h))


ADGI_PACK_RG9, ADGI_PACK_B8, ADGI_PACK_TAU13, ADGI_PACK_TAU2_13 = 0, 1, 2, 3


def pack_channel(values, channel):
    """Packed round trip of a CUDA float32 tensor through one channel
    (adgi_pack_channel): returns (codes int32 tensor, decoded float32 tensor)."""
    import torch
    x = values.contiguous()
    assert x.is_cuda and x.dtype == torch.float32
    codes = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    dec = torch.empty_like(x)
    _check(lib().adgi_pack_channel(C.c_void_p(x.data_ptr()), C.c_int64(x.numel()), C.c_int32(int(channel)),
                                   C.c_void_p(codes.data_ptr()), C.c_void_p(dec.data_ptr()),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return codes, dec


def volume_for_scene(scene, storage=ADGI_FP32, max_rays=None, seed=1, debug=False,
                     irr_res=8, depth_res=16, hysteresis=0.97, **kw) -> Volume:
    """Create a volume on a ``scenes.Scene``'s grid and upload its frame-0 scene."""
    if max_rays is None:
        max_rays = 1 << 20
    vol = Volume(scene.grid_origin, scene.grid_spacing, scene.grid_dims, irr_res=irr_res,
                 depth_res=depth_res, storage=storage, hysteresis=hysteresis,
                 max_rays_per_frame=max_rays, seed=seed, debug=debug, **kw)
    vol.update_scene(scene.positions, scene.indices, scene.albedo, scene.light_positions(0),
                     scene.light_intensity, scene.sky)
    return vol


def _texel_buffers(d, P) -> dict:
    gi, gd = d.irr_res, d.depth_res
    return {"irradiance": np.zeros((P, gi, gi, 3), np.float32),
            "depth": np.zeros((P, gd, gd, 2), np.float32),
            "irr_count": np.zeros((P, gi - 2, gi - 2), np.uint8),
            "depth_count": np.zeros((P, gd - 2, gd - 2), np.uint8),
            "rays_per_probe": np.zeros(P, np.int32),
            "score": np.zeros(P, np.int64)}


class Server:
    """Many probe volumes on one GPU: per-stream frame requests, HBM
    admission by device footprint, eviction to host snapshots (adgi_server_*).

    allocator=None lets the server pool device blocks itself (re-admission
    then allocates nothing); "torch" routes them through torch's allocator."""

    def __init__(self, hbm_budget_bytes, max_inflight=4, allocator=None):
        d = ServerDesc(int(hbm_budget_bytes), int(max_inflight), 0)
        self._alloc = _torch_allocator() if allocator == "torch" else allocator
        h = C.c_void_p()
        _check_server(lib().adgi_server_create(C.byref(d), C.byref(self._alloc) if self._alloc else None,
                                               C.byref(h)))
        self.h = h
        self._streams = []

    @staticmethod
    def now_ns() -> int:
        return int(lib().adgi_server_now_ns())

    def add_stream(self, scene, budget, n_min=8, n_max=2048, storage=ADGI_FP32, seed=1,
                   hysteresis=0.97, beta=5.0, mu=2, theta=8) -> int:
        d = StreamDesc()
        v = d.volume
        v.origin[:] = [float(x) for x in scene.grid_origin]
        v.spacing[:] = [float(x) for x in scene.grid_spacing]
        v.dims[:] = [int(x) for x in scene.grid_dims]
        v.irr_res, v.depth_res, v.storage = 8, 16, int(storage)
        v.hysteresis, v.tau_max = float(hysteresis), TAU_MAX
        v.max_rays_per_frame = int(budget)
        v.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        v.flags = 0
        pos = np.ascontiguousarray(scene.positions, np.float32).reshape(-1, 3)
        idx = np.ascontiguousarray(scene.indices, np.int32).reshape(-1, 3)
        alb = np.ascontiguousarray(scene.albedo, np.float32).reshape(-1, 3)
        lp = np.ascontiguousarray(scene.light_positions(0), np.float32).reshape(-1, 3)
        li = np.ascontiguousarray(scene.light_intensity, np.float32).reshape(-1, 3)
        sd = d.scene
        sd.positions, sd.num_vertices = _ptr(pos), pos.shape[0]
        sd.indices, sd.num_triangles = _ptr(idx), idx.shape[0]
        sd.albedo = _ptr(alb)
        sd.light_pos, sd.light_intensity, sd.num_lights = _ptr(lp), _ptr(li), lp.shape[0]
        sd.sky[:] = [float(x) for x in scene.sky]
        sd.mode = ADGI_SCENE_REBUILD
        d.params = UpdateParams(0, 1, int(budget), int(n_min), int(n_max), 0, float(beta), int(mu),
                                int(theta), 0)
        sid = C.c_int32()
        _check_server(lib().adgi_server_add_stream(self.h, C.byref(d), C.byref(sid)))
        self._streams.append((scene, v))
        return int(sid.value)

    def set_budget(self, hbm_budget_bytes):
        _check_server(lib().adgi_server_set_budget(self.h, int(hbm_budget_bytes)))

    def stream_info(self, sid) -> dict:
        fb, res, fd = C.c_int64(), C.c_int32(), C.c_int32()
        _check_server(lib().adgi_server_stream_info(self.h, int(sid), C.byref(fb), C.byref(res),
                                                    C.byref(fd)))
        return {"footprint_bytes": int(fb.value), "resident": bool(res.value),
                "frames_done": int(fd.value)}

    def submit(self, sid, light_pos, arrival_ns=None):
        lp = np.ascontiguousarray(light_pos, np.float32).reshape(-1, 3)
        t = self.now_ns() if arrival_ns is None else int(arrival_ns)
        _check_server(lib().adgi_server_submit(self.h, int(sid), _ptr(lp), t))

    def progress(self) -> int:
        n = C.c_int32()
        _check_server(lib().adgi_server_progress(self.h, C.byref(n)))
        return int(n.value)

    def drain(self):
        _check_server(lib().adgi_server_drain(self.h))

    def stats(self) -> dict:
        st = ServerStats()
        _check_server(lib().adgi_server_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def latencies(self) -> np.ndarray:
        n = C.c_int64()
        _check_server(lib().adgi_server_latencies(self.h, None, 0, C.byref(n)))
        out = np.zeros(max(int(n.value), 1), np.float64)
        _check_server(lib().adgi_server_latencies(self.h, _ptr(out), out.size, C.byref(n)))
        return out[:int(n.value)]

    def read_stream(self, sid) -> dict:
        scene, v = self._streams[sid]
        P = int(np.prod([int(x) for x in v.dims]))
        out = _texel_buffers(v, P)
        rb = ProbeReadback()
        for k, a in out.items():
            setattr(rb, k, _ptr(a))
        _check_server(lib().adgi_server_read_stream(self.h, int(sid), C.byref(rb)))
        return out

    def destroy(self):
        if getattr(self, "h", None) and self.h.value:
            lib().adgi_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        self.destroy()
