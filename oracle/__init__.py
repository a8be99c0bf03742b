"""FP64 CPU oracle of the adaptive probe-update path (ctypes wrapper).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. It shares no code with
the GPU library ``paper_2301_05125_amd``; the two meet only on the seeded
inputs of ``scenes``.

The arithmetic lives in ``adgi_oracle.c`` (plain C, double precision, OpenMP
over rays/probes); this module only marshals numpy arrays and sequences the
per-frame steps in the order of the paper's frame: pilot rays and change
detection (Sec. 4.1-4.4), the ray budget, then trace + shade + moving-average
update of each probe's texels (Alg. ApproxAlgo, Alg. MovingAvgUpdate).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import time
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "adgi_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Tol(C.Structure):
    _fields_ = [("hit_rel", C.c_double), ("edge_rel", C.c_double), ("edge_abs", C.c_double),
                ("graze", C.c_double), ("bin_eps", C.c_double), ("q10_rel", C.c_double),
                ("q10_abs", C.c_double), ("cos_eps", C.c_double)]


class Hit(C.Structure):
    _fields_ = [("t", C.c_double), ("tri", C.c_int32), ("front", C.c_int32), ("tie", C.c_int32)]


class Ray(C.Structure):
    _fields_ = [("rgb", C.c_double * 3), ("t", C.c_double), ("tri", C.c_int32),
                ("front", C.c_int32), ("shadow", C.c_uint8), ("hit_tie", C.c_int32),
                ("shadow_tie", C.c_int32)]


class Counts(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "hit_ties", "shadow_ties", "bin_ties", "q10_ties",
        "hit_mismatch", "shadow_mismatch", "bin_mismatch", "q10_mismatch",
        "rays", "shadow_rays", "chain_ties", "chain_mismatch")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("dims", C.c_int32 * 3), ("s", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        srcs = [os.path.join(_HERE, n) for n in ("adgi_oracle.c", "adgi_oracle.h")]
        if not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(x) for x in srcs):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        d3 = C.POINTER(C.c_double)
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_key.restype = C.c_uint64
        L.orc_key.argtypes = [C.c_uint64] * 5
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_frame_rotation.argtypes = [C.c_uint64, C.c_int32, P]
        L.orc_sf_dir.argtypes = [C.c_int32, C.c_int32, P, P]
        L.orc_ray_point.restype = C.c_int32
        L.orc_ray_point.argtypes = [C.c_int32, C.c_int32]
        L.orc_pilot_dir.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_oct_encode.argtypes = [P, P]
        L.orc_oct_decode.argtypes = [P, P]
        L.orc_oct_bin.restype = C.c_int32
        L.orc_oct_bin.argtypes = [P, C.c_int32, C.c_double, P]
        L.orc_border_source.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P]
        L.orc_fold_tile.argtypes = [P, C.c_int32, C.c_int32, P]
        L.orc_default_tol.argtypes = [P]
        L.orc_scene_new.restype = P
        L.orc_scene_new.argtypes = [C.c_int32, P, C.c_int32, P, P, C.c_int32]
        L.orc_scene_free.argtypes = [P]
        L.orc_scene_set_positions.argtypes = [P, P]
        L.orc_scene_set_lights.argtypes = [P, C.c_int32, P, P, P]
        L.orc_scene_bvh_depth.restype = C.c_int32
        L.orc_scene_bvh_depth.argtypes = [P]
        L.orc_closest_hit.argtypes = [P, P, P, P, P]
        L.orc_closest_hit_brute.argtypes = [P, P, P, P, P]
        L.orc_occluded.restype = C.c_int32
        L.orc_occluded.argtypes = [P, P, P, C.c_double, P, P]
        L.orc_shade_ray.argtypes = [P, P, P, C.c_double, P, C.c_int32, C.c_int32, P, P, P]
        L.orc_grid_init.argtypes = [P, P, P, P]
        L.orc_probe_pos.argtypes = [P, C.c_int32, P]
        L.orc_pilots.argtypes = [P, P, C.c_uint64, C.c_int32, C.c_double, P, P, P, P, P, P, P, P, P, P]
        L.orc_pilot_blend.argtypes = [P, C.c_uint64, C.c_int32, C.c_int32, P, P, C.c_int32, C.c_int32,
                                      C.c_double, C.c_double, P, P, P, P, P, P, P, P, P]
        L.orc_detect.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P]
        L.orc_allocate.restype = C.c_int32
        L.orc_allocate.argtypes = [C.c_int32, P, C.c_int64, C.c_int32, C.c_int32, P, P, P]
        L.orc_probe_frame.argtypes = [P, P, C.c_int32, C.c_int32, P, P, C.c_int32, C.c_int32,
                                      C.c_double, C.c_double, C.c_int32] + [P] * 14
        L.orc_probes_frame.argtypes = [P, P, C.c_int32, P, P, P, P, P, C.c_int32, C.c_int32,
                                       C.c_double, C.c_double, C.c_int32, C.c_int32] + [P] * 14
        L.orc_blend_alpha.restype = C.c_double
        L.orc_blend_alpha.argtypes = [C.c_int32, C.c_double]
        L.orc_round_half.restype = C.c_double
        L.orc_round_half.argtypes = [C.c_double]
        L.orc_num_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_pack_encode.restype = C.c_uint32
        L.orc_pack_encode.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int32]
        L.orc_pack_decode.restype = C.c_float
        L.orc_pack_decode.argtypes = [C.c_uint32, C.c_float, C.c_float, C.c_int32]
        L.orc_packed_blend.restype = None
        L.orc_chain_h.restype = C.c_double
        L.orc_chain_frame.restype = None
        L.orc_chain_probes_frame.restype = None
        L.orc_chain_probes_frame.argtypes = [P, P, C.c_int32, P, P, P, P, P, P, C.c_int32, C.c_int32,
                                             C.c_double, C.c_double, C.c_int32] + [P] * 9
        L.orc_dynamic_fd.argtypes = [P, C.c_int32, P, P, P, P]
        L.orc_proxy_dims.argtypes = [P, P]
        L.orc_proxy_of_probe.restype = C.c_int32
        L.orc_proxy_of_probe.argtypes = [P, C.c_int32]
        L.orc_proxy_max.argtypes = [P, P, P]
        L.orc_dyn_chain_frame.argtypes = [P, P, C.c_uint64, C.c_int32, P, P, C.c_int32, P, P, P, P]
        L.orc_octant_texels.restype = C.c_int32
        L.orc_octant_texels.argtypes = [C.c_int32, C.c_int32, P]
        L.orc_texel_centre_dir.argtypes = [C.c_int32, C.c_int32, P]
        L.orc_dyn_ray_count.restype = C.c_int32
        L.orc_dyn_ray_count.argtypes = [C.c_int32, C.c_int32, C.c_uint32]
        L.orc_query_irradiance.argtypes = [P, P, C.c_int32, P, C.c_int32, P, P, P]
        L.orc_dyn_probes_frame.argtypes = [P, P, C.c_int32, P, P, P, P, C.c_int32, C.c_int32, C.c_double,
                                           C.c_double, C.c_int32, P, P, P, P, P, P, P]
        L.orc_chain_dir.restype = None
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be contiguous"
    return a.ctypes.data_as(C.c_void_p)


def default_tol() -> Tol:
    t = Tol()
    lib().orc_default_tol(C.byref(t))
    return t


# ------------------------------------------------------------ primitives

def splitmix64(x: int) -> int:
    return lib().orc_splitmix64(x & 0xFFFFFFFFFFFFFFFF)


def frame_rotation(seed: int, frame: int) -> np.ndarray:
    R = np.zeros(9, np.float32)
    lib().orc_frame_rotation(seed & 0xFFFFFFFFFFFFFFFF, frame, _p(R))
    return R.reshape(3, 3)


def sf_dirs(n: int, R: np.ndarray) -> np.ndarray:
    R = np.ascontiguousarray(R, np.float32).reshape(9)
    out = np.zeros((n, 3))
    d = np.zeros(3)
    for j in range(n):
        lib().orc_sf_dir(j, n, _p(R), _p(d))
        out[j] = d
    return out


def ray_point(j: int, n: int) -> int:
    """Index of the spherical Fibonacci point that ray j of an n-ray probe takes."""
    return int(lib().orc_ray_point(j, n))


def probe_ray_dirs(n: int, R: np.ndarray) -> np.ndarray:
    """Directions of an n-ray probe's rays in ray order: ray j along point
    ray_point(j, n) of the rotated spherical Fibonacci set."""
    pts = sf_dirs(n, R)
    return pts[[ray_point(j, n) for j in range(n)]]


def pilot_dir(seed: int, probe: int, k: int, pair: int) -> np.ndarray:
    d = np.zeros(3)
    lib().orc_pilot_dir(seed & 0xFFFFFFFFFFFFFFFF, probe, k, pair, _p(d))
    return d


def oct_encode(d) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    uv = np.zeros(2)
    lib().orc_oct_encode(_p(d), _p(uv))
    return uv


def oct_decode(uv) -> np.ndarray:
    uv = np.ascontiguousarray(uv, np.float64)
    d = np.zeros(3)
    lib().orc_oct_decode(_p(uv), _p(d))
    return d


def oct_bin(d, r: int, eps: float = 0.0):
    d = np.ascontiguousarray(d, np.float64)
    tie = C.c_int32(0)
    k = lib().orc_oct_bin(_p(d), r, eps, C.byref(tie))
    return int(k), bool(tie.value)


def border_source(X: int, Y: int, r: int):
    sx, sy = C.c_int32(), C.c_int32()
    lib().orc_border_source(X, Y, r, C.byref(sx), C.byref(sy))
    return sx.value, sy.value


def fold_tile(interior: np.ndarray, r: int, c: int) -> np.ndarray:
    interior = np.ascontiguousarray(interior, np.float64)
    tile = np.zeros(((r + 2) * (r + 2) * c,))
    lib().orc_fold_tile(_p(interior), r, c, _p(tile))
    return tile.reshape(r + 2, r + 2, c)


def blend_alpha(n: int, h: float) -> float:
    return lib().orc_blend_alpha(n, h)


def round_half(x: float) -> float:
    return lib().orc_round_half(x)


def pack_encode(v: float, beta: float, gamma: float, bits: int) -> int:
    return int(lib().orc_pack_encode(float(v), float(beta), float(gamma), int(bits)))


def pack_decode(q: int, beta: float, gamma: float, bits: int) -> float:
    return float(lib().orc_pack_decode(int(q), float(beta), float(gamma), int(bits)))


# (beta, gamma, bits) per channel of the packed words
PACK_IRR = ((5.0, 15.0, 9), (5.0, 15.0, 9), (5.0, 15.0, 8))
PACK_DEP = ((5.0, 15.0, 13), (8.0, 20.0, 13))


def unpack_words(words: np.ndarray, channels) -> tuple:
    """Packed words -> (decoded FP32 values [..., C], counts [...])."""
    w = np.asarray(words, np.uint32)
    vals = np.zeros(w.shape + (len(channels),), np.float32)
    shift = 0
    dec = np.vectorize(lambda q, b, g, n: pack_decode(int(q), b, g, n), otypes=[np.float32])
    for c, (b, g, n) in enumerate(channels):
        q = (w >> shift) & ((1 << n) - 1)
        vals[..., c] = dec(q, b, g, n) if w.size else 0
        shift += n
    return vals, (w >> 26).astype(np.uint8)


def packed_alpha_table(hysteresis: float) -> np.ndarray:
    """Step weights max(1/(N+1), 1-h) for N = 0..63, in FP32 as the kernel's table."""
    omh = np.float32(1.0 - float(np.float32(hysteresis)))
    k = np.arange(64, dtype=np.float32)
    return np.maximum(np.float32(1.0) / (k + np.float32(1.0)), omh).astype(np.float32)


def packed_blend(n, ray_base, rec, ibin, dbin, ri, rd, inv_s, tau_max, alpha, irr_words, dep_words):
    """Apply one frame of samples to packed interior words in place (FP32)."""
    n = np.ascontiguousarray(n, np.int32)
    ray_base = np.ascontiguousarray(ray_base, np.int64)
    rec = np.ascontiguousarray(rec, np.float32)
    ibin = np.ascontiguousarray(ibin, np.uint16)
    dbin = np.ascontiguousarray(dbin, np.uint16)
    alpha = np.ascontiguousarray(alpha, np.float32)
    assert irr_words.dtype == np.uint32 and dep_words.dtype == np.uint32
    assert irr_words.flags["C_CONTIGUOUS"] and dep_words.flags["C_CONTIGUOUS"]
    lib().orc_packed_blend(C.c_int32(len(n)), _p(n), _p(ray_base), _p(rec), _p(ibin), _p(dbin),
                           C.c_int32(ri), C.c_int32(rd), C.c_float(inv_s), C.c_float(tau_max),
                           _p(alpha), _p(irr_words), _p(dep_words))


class ChainParams(C.Structure):
    _fields_ = [("chains", C.c_int32), ("steps", C.c_int32), ("burn_in", C.c_int32),
                ("sigma_pos", C.c_double), ("sigma_dir", C.c_double)]


SIGMA_DIR = math.sqrt(math.pi / 256.0)  # the paper's angular step (Sec. 4.8)


def chain_h(grid, qv, irr_prev, r: int, x) -> tuple:
    """(h, nearest probe, tie) of the static chain's target at x = (p, uv)."""
    x = np.ascontiguousarray(x, np.float64)
    qv = np.ascontiguousarray(qv, np.uint16)
    irr_prev = np.ascontiguousarray(irr_prev, np.float64)
    pr, tie = C.c_int32(), C.c_int32()
    h = lib().orc_chain_h(C.byref(grid), _p(qv), _p(irr_prev), C.c_int32(r), _p(x), C.byref(pr), C.byref(tie))
    return float(h), int(pr.value), int(tie.value)


def chain_frame(grid, params: ChainParams, seed: int, frame: int, qv, irr_prev, r: int, state,
                init: bool, hint_accept=None, counts=None) -> dict:
    """One frame of every chain (state [C][5] updated in place)."""
    C_, M, K = params.chains, params.steps, params.burn_in
    S = max(M - K - 1, 0)
    qv = np.ascontiguousarray(qv, np.uint16)
    irr_prev = np.ascontiguousarray(irr_prev, np.float64)
    assert state.dtype == np.float64 and state.flags["C_CONTIGUOUS"] and state.shape == (C_, 5)
    acc = np.zeros(max(C_ * M, 1), np.uint8)
    sp = np.zeros(max(C_ * S, 1), np.int32)
    suv = np.zeros((max(C_ * S, 1), 2), np.float64)
    ha = None if hint_accept is None else np.ascontiguousarray(hint_accept, np.uint8)
    cnt = counts if counts is not None else Counts()
    lib().orc_chain_frame(C.byref(grid), C.byref(params), C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                          C.c_int32(frame), _p(qv), _p(irr_prev), C.c_int32(r), _p(state),
                          C.c_int32(1 if init else 0), _p(ha), _p(acc), _p(sp), _p(suv), C.byref(cnt))
    return {"accept": acc[:C_ * M], "sample_probe": sp[:C_ * S], "sample_uv": suv[:C_ * S]}


def dynamic_fd(grid, mu: int, qv, tv, tr) -> np.ndarray:
    """f_d [P*8] (int64) of every (probe, octant), eq. priorDynamic."""
    P = int(np.prod(np.asarray(grid.dims[:], np.int64)))
    fd = np.zeros(P * 8, np.int64)
    lib().orc_dynamic_fd(C.byref(grid), int(mu), _p(np.ascontiguousarray(qv, np.uint16)),
                         _p(np.ascontiguousarray(tv, np.int32)), _p(np.ascontiguousarray(tr, np.int32)),
                         _p(fd))
    return fd


def proxy_dims(grid) -> tuple:
    pd = np.zeros(3, np.int32)
    lib().orc_proxy_dims(C.byref(grid), _p(pd))
    return tuple(int(x) for x in pd)


def proxy_max(grid, fd) -> np.ndarray:
    """F [Pp*8] (int64): max of f_d over each 3x3x3 proxy, per octant."""
    Pp = int(np.prod(proxy_dims(grid)))
    F = np.zeros(Pp * 8, np.int64)
    lib().orc_proxy_max(C.byref(grid), _p(np.ascontiguousarray(fd, np.int64)), _p(F))
    return F


def dyn_chain_frame(grid, params: ChainParams, seed: int, frame: int, F, state, init: bool,
                    hint_accept=None, counts=None) -> dict:
    """One frame of every dynamic chain (state [C][5] in place) -> marks [Pp*8]."""
    C_, M = params.chains, params.steps
    assert state.dtype == np.float64 and state.flags["C_CONTIGUOUS"] and state.shape == (C_, 5)
    F = np.ascontiguousarray(F, np.int64)
    mark = np.zeros(F.shape[0], np.uint8)
    acc = np.zeros(max(C_ * M, 1), np.uint8)
    ha = None if hint_accept is None else np.ascontiguousarray(hint_accept, np.uint8)
    cnt = counts if counts is not None else Counts()
    lib().orc_dyn_chain_frame(C.byref(grid), C.byref(params), seed & 0xFFFFFFFFFFFFFFFF, int(frame), _p(F),
                              _p(state), 1 if init else 0, _p(ha), _p(acc), _p(mark), C.byref(cnt))
    return {"accept": acc[:C_ * M], "mark": mark}


def octant_texels(r: int, k: int) -> np.ndarray:
    n = lib().orc_octant_texels(r, k, None)
    out = np.zeros(max(n, 1), np.int32)
    lib().orc_octant_texels(r, k, _p(out))
    return out[:n]


def texel_centre_dir(r: int, t: int) -> np.ndarray:
    d = np.zeros(3)
    lib().orc_texel_centre_dir(r, t, _p(d))
    return d


def dyn_ray_counts(grid, mark, irr_res: int, depth_res: int) -> np.ndarray:
    """Dynamic rays of every probe (probe order) given the proxy marks."""
    P = int(np.prod(np.asarray(grid.dims[:], np.int64)))
    mark = np.asarray(mark, np.uint8).reshape(-1, 8)
    bits = (mark.astype(np.uint32) << np.arange(8, dtype=np.uint32)).sum(axis=1)
    per_mask = np.array([lib().orc_dyn_ray_count(irr_res, depth_res, m) for m in range(256)], np.int64)
    px = np.array([lib().orc_proxy_of_probe(C.byref(grid), i) for i in range(P)], np.int64)
    return per_mask[bits[px]]


def query_irradiance(grid, irr_tiles, dep_tiles, points, normals) -> np.ndarray:
    """Irradiance [K][3] at points [K][3] with normals [K][3] from full tiles."""
    irr = np.ascontiguousarray(irr_tiles, np.float64)
    dep = np.ascontiguousarray(dep_tiles, np.float64)
    pts = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(normals, np.float64).reshape(-1, 3)
    out = np.zeros((pts.shape[0], 3))
    row = np.zeros(3)
    for k in range(pts.shape[0]):
        lib().orc_query_irradiance(C.byref(grid), _p(irr), irr.shape[1], _p(dep), dep.shape[1],
                                   _p(pts[k]), _p(nrm[k]), _p(row))
        out[k] = row
    return out


def chain_order(sample_probe: np.ndarray, P: int):
    """Samples grouped by probe, ascending sample index within a probe:
    (permutation, samples per probe, first sample of each probe)."""
    perm = np.argsort(np.asarray(sample_probe), kind="stable")
    n = np.bincount(np.asarray(sample_probe, np.int64), minlength=P).astype(np.int32)
    base = np.concatenate([[0], np.cumsum(n, dtype=np.int64)])[:-1]
    return perm, n, base


def allocate(score: np.ndarray, budget: int, n_min: int, n_max: int):
    """Integer budget allocation. Returns (n[P] int32, offsets[P+1] int64, lambda*)."""
    score = np.ascontiguousarray(score, np.int64)
    P = score.shape[0]
    n = np.zeros(P, np.int32)
    off = np.zeros(P + 1, np.int64)
    lam = C.c_uint32(0)
    rc = lib().orc_allocate(P, _p(score), int(budget), n_min, n_max, _p(n), _p(off), C.byref(lam))
    if rc != 0:
        raise ValueError("budget below P * n_min or bad bounds")
    return n, off, int(lam.value)


class OracleScene:
    """Triangles + lights in FP64 with the oracle's own BVH (or brute force)."""

    def __init__(self, positions, indices, albedo, use_bvh: bool = True):
        self.positions = np.ascontiguousarray(positions, np.float32)
        self.indices = np.ascontiguousarray(indices, np.int32)
        self.albedo = np.ascontiguousarray(albedo, np.float32)
        self.ptr = lib().orc_scene_new(self.positions.shape[0], _p(self.positions),
                                       self.indices.shape[0], _p(self.indices), _p(self.albedo),
                                       1 if use_bvh else 0)

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_scene_free(self.ptr)
            self.ptr = None

    def set_positions(self, positions):
        self.positions = np.ascontiguousarray(positions, np.float32)
        lib().orc_scene_set_positions(self.ptr, _p(self.positions))

    def set_lights(self, lpos, lint, sky):
        self._lp = np.ascontiguousarray(lpos, np.float32).reshape(-1, 3)
        self._li = np.ascontiguousarray(lint, np.float32).reshape(-1, 3)
        self._sky = np.ascontiguousarray(sky, np.float32).reshape(3)
        lib().orc_scene_set_lights(self.ptr, self._lp.shape[0], _p(self._lp), _p(self._li),
                                   _p(self._sky))

    @property
    def bvh_depth(self) -> int:
        return lib().orc_scene_bvh_depth(self.ptr)

    def closest_hit(self, o, d, tol: Optional[Tol] = None, brute: bool = False) -> Hit:
        o = np.ascontiguousarray(o, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        h = Hit()
        fn = lib().orc_closest_hit_brute if brute else lib().orc_closest_hit
        fn(self.ptr, _p(o), _p(d), C.byref(tol) if tol is not None else None, C.byref(h))
        return h

    def occluded(self, o, d, tmax: float, tol: Optional[Tol] = None):
        o = np.ascontiguousarray(o, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        tie = C.c_int32(0)
        r = lib().orc_occluded(self.ptr, _p(o), _p(d), tmax,
                               C.byref(tol) if tol is not None else None, C.byref(tie))
        return bool(r), bool(tie.value)

    def shade(self, o, d, spacing_diag: float, tol: Optional[Tol] = None) -> Ray:
        o = np.ascontiguousarray(o, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        r = Ray()
        lib().orc_shade_ray(self.ptr, _p(o), _p(d), spacing_diag,
                            C.byref(tol) if tol is not None else None, -2, -1, C.byref(r),
                            None, None)
        return r


def make_grid(origin, spacing, dims) -> Grid:
    g = Grid()
    o = np.ascontiguousarray(origin, np.float32)
    s = np.ascontiguousarray(spacing, np.float32)
    d = np.ascontiguousarray(dims, np.int32)
    lib().orc_grid_init(C.byref(g), _p(o), _p(s), _p(d))
    return g


TAU_MAX = (math.exp(5.0) - 1.0) / 15.0


class OracleVolume:
    """The per-frame probe update in FP64, state kept for a set of probes.

    ``probes`` selects which probes' texels are tracked (all by default);
    detection and allocation always cover the whole grid because the budget
    couples every probe.
    """

    def __init__(self, scene, irr_res: int = 8, depth_res: int = 16,
                 hysteresis: float = 0.97, tau_max: float = TAU_MAX, seed: int = 1,
                 fp16: bool = False, probes: Optional[np.ndarray] = None,
                 use_bvh: bool = True, tol: Optional[Tol] = None, gather: bool = False):
        self.sc = scene
        self.scene = OracleScene(scene.positions, scene.indices, scene.albedo, use_bvh=use_bvh)
        self.grid = make_grid(scene.grid_origin, scene.grid_spacing, scene.grid_dims)
        self.P = int(np.prod(scene.grid_dims.astype(np.int64)))
        self.irr_res, self.depth_res = irr_res, depth_res
        # parameters arrive as FP32 and are promoted
        self.h = float(np.float32(hysteresis))
        self.tau_max = float(np.float32(tau_max))
        self.seed = seed
        self.fp16 = bool(fp16)
        self.gather = bool(gather)  # DDGI's cosine-weighted gather instead of per-sample updates
        self.tol = tol if tol is not None else default_tol()
        self.probes = (np.arange(self.P, dtype=np.int32) if probes is None
                       else np.ascontiguousarray(probes, np.int32))
        nq = self.probes.shape[0]
        ri, rd = irr_res - 2, depth_res - 2
        self.irr = np.zeros((nq, ri * ri * 3))
        self.irr_n = np.zeros((nq, ri * ri), np.uint8)
        self.dep = np.zeros((nq, rd * rd * 2))
        self.dep_n = np.zeros((nq, rd * rd), np.uint8)
        self.qv_prev = np.zeros(self.P * 8, np.uint16)
        self.qr_prev = np.zeros(self.P * 8, np.uint16)
        self.tv = np.zeros(self.P * 8, np.int32)
        self.tr = np.zeros(self.P * 8, np.int32)
        self.score = np.zeros(self.P, np.int64)
        self.qv_odd = np.zeros(self.P * 8, np.uint16)  # codes of the last frame that ran detection
        self.counts = Counts()

    def set_frame_inputs(self, frame: int):
        sc = self.sc
        if sc.anim_vertices and frame > 0:
            self.scene.set_positions(sc.positions_at(frame))
        self.scene.set_lights(sc.light_positions(frame), sc.light_intensity, sc.sky)

    def pilots(self, frame: int, beta: float = 5.0, hint_qv=None, hint_qr=None, counts=None,
               hint_tri=None, hint_shadow=None, records: bool = False):
        """Pilot codes (Qv, Qr) of every probe and octant; ties and
        mismatches against the hints go to ``counts`` (default: the running
        totals). With ``records`` also each pilot's radiance [P*8, 3] and
        hit distance [P*8]."""
        qv = np.zeros(self.P * 8, np.uint16)
        qr = np.zeros(self.P * 8, np.uint16)
        prgb = np.zeros((self.P * 8, 3)) if records else None
        pt = np.zeros(self.P * 8) if records else None
        h_tri = None if hint_tri is None else np.ascontiguousarray(hint_tri, np.int32)
        h_sh = None if hint_shadow is None else np.ascontiguousarray(hint_shadow, np.uint8)
        lib().orc_pilots(self.scene.ptr, C.byref(self.grid), self.seed & 0xFFFFFFFFFFFFFFFF,
                         frame, float(np.float32(beta)), C.byref(self.tol),
                         _p(hint_qv), _p(hint_qr), _p(h_tri), _p(h_sh), _p(qv), _p(qr), _p(prgb), _p(pt),
                         C.byref(counts if counts is not None else self.counts))
        if records:
            return qv, qr, prgb, pt
        return qv, qr

    def pilot_blend(self, frame: int, prgb, pt, hint_ibin=None, hint_dbin=None, counts=None):
        """Pilot reuse (Sec. 4.4): the tracked probes' 8 pilot samples into
        their texels, in octant order."""
        h_ib = None if hint_ibin is None else np.ascontiguousarray(hint_ibin, np.uint16)
        h_db = None if hint_dbin is None else np.ascontiguousarray(hint_dbin, np.uint16)
        lib().orc_pilot_blend(C.byref(self.grid), self.seed & 0xFFFFFFFFFFFFFFFF, frame,
                              self.probes.shape[0], _p(self.probes), C.byref(self.tol), self.irr_res,
                              self.depth_res, self.h, self.tau_max, _p(np.ascontiguousarray(prgb)),
                              _p(np.ascontiguousarray(pt)), _p(h_ib), _p(h_db), _p(self.irr), _p(self.irr_n),
                              _p(self.dep), _p(self.dep_n),
                              C.byref(counts if counts is not None else self.counts))

    def detect(self, frame: int, qv, qr, theta: int = 8, mu: int = 2):
        lib().orc_detect(C.byref(self.grid), frame, theta, mu, _p(qv), _p(qr),
                         _p(self.qv_prev), _p(self.qr_prev), _p(self.tv), _p(self.tr),
                         _p(self.score))
        return self.score.copy()

    def update(self, frame: int, adaptive: bool, budget: int = 0, n_min: int = 8,
               n_max: int = 2048, n_uniform: int = 64, beta: float = 5.0, mu: int = 2,
               theta: int = 8, hints: Optional[dict] = None, keep_rays: bool = False,
               pilot_reuse: bool = False) -> dict:
        """One frame. ``hints`` holds the GPU's discrete decisions (lockstep).
        ``pilot_reuse``: on the first frame of each pilot pair the pilots'
        samples also update the caches, before the frame's probe rays
        (Sec. 4.4)."""
        hints = hints or {}
        t0 = time.perf_counter()
        self.set_frame_inputs(frame)
        out = {}
        secs = {"scene": time.perf_counter() - t0, "pilots": 0.0, "detect_allocate": 0.0,
                "probes": 0.0}
        cnt = Counts()
        if adaptive:
            t0 = time.perf_counter()
            reuse = pilot_reuse and frame % 2 == 0
            qv, qr, prgb, pt = self.pilots(frame, beta, hints.get("qv"), hints.get("qr"), counts=cnt,
                                           hint_tri=hints.get("pilot_tri"),
                                           hint_shadow=hints.get("pilot_shadow"), records=True)
            if reuse:
                self.pilot_blend(frame, prgb, pt, hints.get("pilot_ibin"), hints.get("pilot_dbin"), counts=cnt)
            out.update(pilot_rgb=prgb, pilot_t=pt)
            t1 = time.perf_counter()
            score = self.detect(frame, qv, qr, theta, mu)
            n, off, lam = allocate(score, budget, n_min, n_max)
            secs["pilots"], secs["detect_allocate"] = t1 - t0, time.perf_counter() - t1
            out.update(qv=qv, qr=qr, score=score, lam=lam)
        else:
            n = np.full(self.P, n_uniform, np.int32)
            off = np.concatenate([[0], np.cumsum(n, dtype=np.int64)])
        out.update(n=n, offsets=off)
        R = frame_rotation(self.seed, frame)
        out["R"] = R
        Rf = np.ascontiguousarray(R.reshape(9), np.float32)
        nq = self.probes.shape[0]
        n_sel = np.ascontiguousarray(n[self.probes], np.int32)
        base_global = off[self.probes]
        # outputs and hints are addressed in a compact per-subset ray space
        local_base = np.concatenate([[0], np.cumsum(n_sel, dtype=np.int64)])
        total = int(local_base[-1])
        ray_base = np.ascontiguousarray(local_base[:-1], np.int64)

        def gather(name, dtype):
            a = hints.get(name)
            if a is None:
                return None
            a = np.asarray(a)
            idx = np.concatenate([np.arange(b, b + k, dtype=np.int64)
                                  for b, k in zip(base_global, n_sel)]) if total else np.zeros(0, np.int64)
            return np.ascontiguousarray(a[idx], dtype)

        h_tri = gather("hit_tri", np.int32)
        h_sh = gather("shadow_bits", np.uint8)
        h_ib = gather("irr_bin", np.uint16)
        h_db = gather("depth_bin", np.uint16)
        rays = np.zeros((max(total, 1), 4)) if keep_rays else None
        tri = np.zeros(max(total, 1), np.int32) if keep_rays else None
        sh = np.zeros(max(total, 1), np.uint8) if keep_rays else None
        ib = np.zeros(max(total, 1), np.uint16) if keep_rays else None
        db = np.zeros(max(total, 1), np.uint16) if keep_rays else None
        t0 = time.perf_counter()
        lib().orc_probes_frame(
            self.scene.ptr, C.byref(self.grid), nq, _p(self.probes), _p(n_sel), _p(ray_base),
            _p(Rf), C.byref(self.tol), self.irr_res, self.depth_res, self.h, self.tau_max,
            1 if self.fp16 else 0, 1 if self.gather else 0, _p(h_tri), _p(h_sh), _p(h_ib), _p(h_db),
            _p(self.irr), _p(self.irr_n), _p(self.dep), _p(self.dep_n),
            _p(rays), _p(tri), _p(sh), _p(ib), _p(db), C.byref(cnt))
        secs["probes"] = time.perf_counter() - t0
        out["seconds"] = secs
        for name, _ in Counts._fields_:
            setattr(self.counts, name, getattr(self.counts, name) + getattr(cnt, name))
        out["counts"] = cnt.as_dict()
        if keep_rays:
            out.update(rays=rays[:total], tri=tri[:total], shadow=sh[:total], irr_bin=ib[:total],
                       depth_bin=db[:total], ray_base=ray_base)
        return out

    def chain_update(self, frame: int, params: "ChainParams", state: np.ndarray, init: bool,
                     beta: float = 5.0, hints: Optional[dict] = None, mu: int = 2, theta: int = 8,
                     dyn: Optional["ChainParams"] = None, dyn_state: Optional[np.ndarray] = None,
                     dyn_init: bool = False, h_dyn: float = 0.91, pilot_reuse: bool = False) -> dict:
        """One chain frame: pilots (for f_v), detection (triggers and scores
        kept current), one frame of every static chain against the previous
        frame's irradiance, each sample's two rays blended into its nearest
        probe in sample order; with ``dyn``, the dynamic chains on the 3x3x3
        proxies of f_d mark (proxy, octant) pairs, static samples at probes
        with a dynamic component trace through texel centres, and every
        probe of a marked proxy then updates the octant's texels through
        their centres with hysteresis ``h_dyn``. Tracks every probe.
        ``state`` / ``dyn_state`` [C][5] are updated in place; ``hints`` may
        hold the GPU's qv/qr codes, accept decisions and per-ray decisions
        (sample rays in the GPU's sorted order, then the dynamic rays)."""
        assert self.probes.shape[0] == self.P, "chain frames need every probe tracked"
        hints = hints or {}
        self.set_frame_inputs(frame)
        cnt = Counts()
        qv, qr, prgb, pt = self.pilots(frame, beta, hints.get("qv"), hints.get("qr"), counts=cnt,
                                       hint_tri=hints.get("pilot_tri"), hint_shadow=hints.get("pilot_shadow"),
                                       records=True)
        self.detect(frame, qv, qr, theta, mu)
        if frame & 1:
            self.qv_odd = qv.copy()
        ri, rd = self.irr_res - 2, self.depth_res - 2
        # the guide reads the previous frame's irradiance, before this frame's
        # pilot samples enter the caches
        irr_prev = self.irr.copy()
        if pilot_reuse and frame % 2 == 0:
            self.pilot_blend(frame, prgb, pt, hints.get("pilot_ibin"), hints.get("pilot_dbin"), counts=cnt)
        out = chain_frame(self.grid, params, self.seed, frame, qv, irr_prev, ri, state, init,
                          hints.get("accept"), cnt)
        perm, n, base = chain_order(out["sample_probe"], self.P)
        suv = np.ascontiguousarray(out["sample_uv"][perm])
        S2 = 2 * len(perm)
        quant = None
        if dyn is not None:
            self.h_dyn = float(np.float32(h_dyn))
            fd = dynamic_fd(self.grid, mu, self.qv_odd, self.tv, self.tr)
            F = proxy_max(self.grid, fd)
            dout = dyn_chain_frame(self.grid, dyn, self.seed, frame, F, dyn_state, dyn_init,
                                   hints.get("dyn_accept"), cnt)
            quant = np.ascontiguousarray(self.score > 0, np.uint8)
            out.update(F=F, fd=fd, mark=dout["mark"], dyn_accept=dout["accept"])

        def h(name, dtype, lo, hi):
            a = hints.get(name)
            return None if a is None else np.ascontiguousarray(np.asarray(a)[lo:hi], dtype)

        lib().orc_chain_probes_frame(
            self.scene.ptr, C.byref(self.grid), self.P, _p(self.probes), _p(n), _p(base), _p(suv),
            _p(quant), C.byref(self.tol), self.irr_res, self.depth_res, self.h, self.tau_max,
            1 if (self.fp16 and dyn is None) else 0, _p(h("hit_tri", np.int32, 0, S2)),
            _p(h("shadow_bits", np.uint8, 0, S2)), _p(h("irr_bin", np.uint16, 0, S2)),
            _p(h("depth_bin", np.uint16, 0, S2)), _p(self.irr), _p(self.irr_n), _p(self.dep),
            _p(self.dep_n), C.byref(cnt))
        if dyn is not None:
            nd = dyn_ray_counts(self.grid, out["mark"], self.irr_res, self.depth_res)
            dbase = np.ascontiguousarray(np.concatenate([[0], np.cumsum(nd)])[:-1], np.int64)
            R = int(nd.sum())
            lib().orc_dyn_probes_frame(
                self.scene.ptr, C.byref(self.grid), self.P, _p(self.probes), _p(out["mark"]), _p(dbase),
                C.byref(self.tol), self.irr_res, self.depth_res, self.h_dyn, self.tau_max,
                1 if self.fp16 else 0, _p(h("hit_tri", np.int32, S2, S2 + R)),
                _p(h("shadow_bits", np.uint8, S2, S2 + R)), _p(self.irr), _p(self.irr_n), _p(self.dep),
                _p(self.dep_n), C.byref(cnt))
            out.update(dyn_rays=nd, dyn_offsets=np.concatenate([dbase, [R]]))
        for name, _ in Counts._fields_:
            setattr(self.counts, name, getattr(self.counts, name) + getattr(cnt, name))
        out.update(qv=qv, qr=qr, n=n, offsets=np.concatenate([base, [len(perm)]]), perm=perm,
                   counts=cnt.as_dict(), score=self.score.copy())
        return out

    # views in the library's readback layout
    def irradiance_tiles(self) -> np.ndarray:
        ri = self.irr_res - 2
        return np.stack([fold_tile(t, ri, 3) for t in self.irr])

    def depth_tiles(self) -> np.ndarray:
        rd = self.depth_res - 2
        return np.stack([fold_tile(t, rd, 2) for t in self.dep])
