/* adgi.h - C ABI of the MI355X probe-update library.
 *
 * The library keeps a uniform grid of light probes up to date each frame, as
 * in the adaptive probe update of "Adaptive Dynamic Global Illumination"
 * (Datta, Goli & Zhang, arXiv 2301.05125):
 *
 *   1. pilot rays, one per octant of every probe, measure probe visibility
 *      f_v = exp(-2t/s) (eq. ProbeVis) and incoming radiance
 *      f_r = min(lum, beta)/beta (Sec. 4.1.3); their temporal change, passed
 *      through a decaying trigger and a 5x5x5 spatial sum (Sec. 4.1.4-4.1.5),
 *      is composed as f_v (f_dv + mu f_dr) (eq. priorDynamic) into an integer
 *      score per probe;
 *   2. a user-set total ray budget is split over the probes in proportion to
 *      their scores (the paper fixes the samples per frame and lets its guide
 *      place them, Sec. 3.3), each probe getting between n_min and n_max rays;
 *   3. every probe traces its rays (a randomly rotated spherical Fibonacci
 *      set, as DDGI's rotated spiral, Sec. 3.1) against a triangle BVH, with
 *      direct light and shadow rays at each hit;
 *   4. each sample updates the octahedral irradiance texel and the
 *      depth-moment (visibility) texel it falls in with the moving average of
 *      Alg. MovingAvgUpdate (Alg. ApproxAlgo, Sec. 4.5-4.7).
 * With adaptive = 0 every probe traces n_uniform rays and steps 1-2 are
 * skipped (the uniform DDGI-style update). With adaptive = ADGI_MODE_CHAIN
 * the rays are placed by static Metropolis chains instead of steps 2-3
 * (Sec. 3.2-3.3, Alg. MarkovChainMT and MetropolisStep, Sec. 4.8): see
 * adgi_update_params.
 *
 * Conventions
 *   - Probe i sits at origin + (x, y, z) * spacing with
 *     i = x + dims[0] * (y + dims[1] * z).
 *   - s = |spacing|_2 is the voxel diagonal (the length eq. ProbeVis
 *     normalises distances by); depth texels store tau = min(t/s, tau_max)
 *     and tau^2.
 *   - Texel tiles are res x res with a one-texel border copied across the
 *     octahedral map's edges; the interior is (res-2) x (res-2). Direction d
 *     falls in the interior texel of its octahedral coordinates (Cigolle et
 *     al. 2014), row = v, column = u.
 *   - All functions return an adgi_status; on any error nothing has been
 *     enqueued, the volume and every output are unchanged, and
 *     adgi_last_error() describes the failure. A device error is sticky: every
 *     later call on that volume returns ADGI_ERR_DEVICE until it is destroyed.
 *   - A volume is not thread-safe. Distinct volumes may be used from distinct
 *     threads and overlap on the device.
 *   - Pointers marked "host" are CPU memory owned by the caller and only read
 *     or written during the call. All device memory belongs to the library.
 */
#ifndef ADGI_H
#define ADGI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adgi_volume adgi_volume;

typedef enum {
  ADGI_OK = 0,
  ADGI_ERR_INVALID_ARG = -1,   /* a descriptor or argument is out of range        */
  ADGI_ERR_OUT_OF_MEMORY = -2, /* the allocator returned NULL                     */
  ADGI_ERR_BUDGET = -3,        /* budget < P*n_min, n_min < 1 or n_max < n_min,
                                  or the rays would exceed max_rays_per_frame     */
  ADGI_ERR_NO_SCENE = -4,      /* update_probes before any update_scene           */
  ADGI_ERR_TOPOLOGY = -5,      /* REFIT with a different vertex/triangle count    */
  ADGI_ERR_DEVICE = -6         /* a HIP call failed; sticky until destroy         */
} adgi_status;

/* Texel storage. ADGI_PACKED is the paper's 32-bit texel (Sec. 4.5-4.6, eq.
 * rgbEnc, App. B): irradiance R9 G9 B8 + count N6, each colour channel
 * u = min(ln(15 v + 1), 5) / 5 stored as floor(u (2^bits - 1)); depth tau13 +
 * tau^2_13 + N6 with (beta, gamma) = (5, 15) and (8, 20); counts saturate at
 * 63; every sample decodes, updates and re-encodes its texel (binary32
 * arithmetic). Needs tiles 8/16 or 16/16. */
enum { ADGI_FP32 = 0, ADGI_FP16 = 1, ADGI_PACKED = 2 };
enum { ADGI_SCENE_REBUILD = 0, ADGI_SCENE_REFIT = 1 };      /* scene update mode */
/* Volume flags. ADGI_STATIC_SCRATCH: the volume allocates no frame scratch
 * (pair lists, hit points, detection sums, allocation partials, blend order,
 * frame counters: about 60 bytes per ray of max(max_rays_per_frame, 8 P)),
 * and its frames run only through adgi_update_probes_static; needs
 * max_chains = 0. */
enum { ADGI_DEBUG_ARRAYS = 1u << 0, ADGI_STATIC_SCRATCH = 1u << 1 };
enum { ADGI_MAX_LIGHTS = 8 };
enum { ADGI_MODE_UNIFORM = 0, ADGI_MODE_ADAPTIVE = 1, ADGI_MODE_CHAIN = 2 };  /* params.adaptive */
/* Texel update (volume desc): ADGI_BLEND_SAMPLE, the paper's per-sample
 * moving average into the texel holding each direction (Alg. ApproxAlgo,
 * Alg. MovingAvgUpdate); ADGI_BLEND_GATHER, DDGI's cosine-weighted gather
 * (Majercik et al. 2019; the update Sec. 3.1 describes): every texel takes all
 * of the probe's rays of the frame weighted by max(0, c.d), c its centre
 * direction (depth: that cosine to the 50th power), and their weighted mean
 * enters the texel with a = max(1/(N+1), 1 - h), N counting the frames in
 * which the texel had weight. Gather: ADGI_FP32 / ADGI_FP16, tiles 8/16 or
 * 16/16, budgeted or uniform frames. */
enum { ADGI_BLEND_SAMPLE = 0, ADGI_BLEND_GATHER = 1 };
enum { ADGI_CHAIN_MAX_STEPS = 256 };

/* Device memory provider. alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL; free releases it. Both are called only from
 * create/update_scene/destroy and from adgi_autotune. NULL allocator = hipMalloc. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} adgi_allocator;

typedef struct {
  float origin[3];            /* centre of probe (0,0,0), world units            */
  float spacing[3];           /* > 0                                             */
  int32_t dims[3];            /* >= 1 each; P = product, P <= 2^24               */
  int32_t irr_res;            /* irradiance tile side incl. border, 3..34 (8)    */
  int32_t depth_res;          /* depth tile side incl. border, 3..34 (16)        */
  int32_t storage;            /* ADGI_FP32, ADGI_FP16 or ADGI_PACKED              */
  float hysteresis;           /* h in [0, 1): step = max(1/(N+1), 1-h) (0.97)    */
  float tau_max;              /* depth clamp in units of s ((e^5-1)/15)          */
  int64_t max_rays_per_frame; /* capacity of the per-frame ray buffers, < 2^31   */
  uint64_t seed;              /* seeds the frame rotation and the pilot rays     */
  uint32_t flags;             /* ADGI_DEBUG_ARRAYS keeps per-ray decisions;
                                 ADGI_STATIC_SCRATCH (see the flags above)       */
  int32_t max_chains;         /* 0, or the most Metropolis chains a frame may run
                                 (ADGI_FP32 / ADGI_FP16, tiles 8/16 or 16/16);
                                 allocates the chain state and sample buffers for
                                 max_rays/2 samples                               */
  int32_t blend_mode;         /* ADGI_BLEND_SAMPLE (0) or ADGI_BLEND_GATHER         */
} adgi_volume_desc;

typedef struct {
  const float* positions;     /* host [num_vertices][3]                           */
  int32_t num_vertices;
  const int32_t* indices;     /* host [num_triangles][3], 0 <= index < V          */
  int32_t num_triangles;      /* >= 0 (0 = empty scene: every ray sees the sky)   */
  const float* albedo;        /* host [num_triangles][3]; ignored by REFIT        */
  const float* light_pos;     /* host [num_lights][3]                              */
  const float* light_intensity;/* host [num_lights][3] RGB                         */
  int32_t num_lights;         /* 0..ADGI_MAX_LIGHTS                                */
  float sky[3];               /* radiance of rays that leave the scene            */
  int32_t mode;               /* REBUILD: new triangles, host SAH build.
                                 REFIT: same V and T, positions[vbegin, vend)
                                 changed (only they are uploaded; the others keep
                                 their last uploaded values); the triangles that
                                 touch the range are rebuilt and the boxes refitted
                                 on the device (every triangle on the first REFIT
                                 after a REBUILD).                                */
  int32_t refit_vertex_begin; /* REFIT only; [0, V]                                */
  int32_t refit_vertex_end;   /* REFIT only; [begin, V]                            */
} adgi_scene_desc;

typedef struct {
  int32_t frame;              /* frame index t >= 0; consecutive frames form pairs
                                 (2m, 2m+1) that share pilot directions           */
  int32_t adaptive;           /* 0: n_uniform rays per probe; 1: budgeted          */
  int64_t budget;             /* adaptive: total rays B this frame                 */
  int32_t n_min, n_max;       /* adaptive: per-probe bounds                        */
  int32_t n_uniform;          /* uniform: rays per probe, >= 1                     */
  float beta;                 /* f_r dynamic range (5)                              */
  int32_t mu;                 /* weight of radiance change vs visibility change (2) */
  int32_t theta;              /* trigger decays to 0 in theta detection steps (8)  */
  int32_t sync;               /* 1: wait for completion and fill stats             */
  /* ADGI_MODE_CHAIN (Sec. 3.2-3.3, Sec. 4.8). Chain c's state is a point x = (p, uv):
   * p in the box spanned by the probe centres, uv the octahedral coordinates
   * of a direction. Its target density is h(x) = exp(min(g/f, 1)) f, with
   * f = Qv/1024 the pilot visibility code of this frame in the octant of uv at
   * the probe nearest to p, and g the luminance of that probe's irradiance
   * averaged over the 2x2 interior texels whose cell holds uv, as the
   * previous frame left it. Every frame each chain takes chain_steps
   * Metropolis steps from where it stopped (normal proposals, sigma_pos *
   * spacing per axis and sigma_dir in uv; a proposal outside the domain is
   * rejected; it is accepted when h(x) = 0 or u h(x) <= h(x'), all uniforms
   * from the counter-based stream; a grid axis with one probe has no extent
   * and chains do not move along it). Each step after the first
   * chain_burn_in + 1 emits a sample (nearest probe, uv), so a frame makes
   * S = chain_count (chain_steps - chain_burn_in - 1) samples. A sample
   * traces two rays from its probe's centre: d(uv), shaded with direct light
   * and blended into the irradiance texel of d, and -d, whose distance only
   * is blended into the depth texel of -d. Per-probe lists are the samples
   * in chain-major order. Pilots run as in ADAPTIVE and detection on odd
   * frames; the budget split is skipped. With use_graph, chain frames are
   * captured as graphs too, one per frame parity, captured again when the
   * chain count, lanes, samples or dynamic chain count change. */
  int32_t chain_count;        /* C, 1..max_chains                                  */
  int32_t chain_steps;        /* M, 2..ADGI_CHAIN_MAX_STEPS                        */
  int32_t chain_burn_in;      /* K, 0 <= K <= M - 2                                */
  float chain_sigma_pos;      /* > 0, in units of the grid spacing (0.5)           */
  float chain_sigma_dir;      /* > 0, in octahedral uv units (sqrt(pi/256))        */
  int32_t chain_reset;        /* 1: start every chain from its seeded initial point;
                                 chains also start there on their first frame and
                                 whenever chain_count changes (dynamic chains too) */
  /* Dynamic chains (Sec. 4.9), chain frames only. Probes form virtual proxies
   * of 3x3x3 (the last group along an axis may be smaller). Every (probe,
   * octant) has a dynamic component f_d = Qv (Cv + mu Cr) (eq. priorDynamic:
   * Qv the pilot visibility code and C the 5x5x5 trigger sums of the last
   * detection, which chain frames run as budgeted frames do); F of a proxy
   * and octant is the max over its probes. dyn_chain_count chains walk
   * like the static ones (their own random stream, steps dyn_sigma_pos *
   * spacing and dyn_sigma_dir) on the target h = F[proxy of the nearest
   * probe][octant of uv]; every state past the burn-in with h > 0 marks its
   * (proxy, octant). After the frame's static samples, every probe of a
   * marked proxy updates each irradiance texel of the octant with a shaded
   * ray through the texel's centre and each depth texel of the octant with
   * the distance of a ray through its centre (texel centres belong to an
   * octant by the signs of their octahedral coordinates and |u| + |v| > 1,
   * centres on the diagonal to the upper half), with the step floor
   * 1 - dyn_hysteresis. With dynamic chains on, static samples at probes
   * with score > 0 trace through the centres of their texels. Capacity:
   * 2 S + min(P (ri^2 + rd^2), 27 m min(8 Pp, C_d S_d)) <= max_rays_per_frame,
   * ri, rd the interior sides, m the most texels of one octant in both maps. */
  int32_t dyn_chain_count;    /* 0 (none) or 1..max_chains                         */
  int32_t dyn_chain_steps;    /* 2..ADGI_CHAIN_MAX_STEPS                           */
  int32_t dyn_chain_burn_in;  /* 0..dyn_chain_steps - 2                            */
  float dyn_sigma_pos;        /* > 0 (1.5: three times the static default)         */
  float dyn_sigma_dir;        /* > 0 (6 sqrt(pi/256))                              */
  float dyn_hysteresis;       /* [0, 1) (0.91, Tab. cacheDetails)                   */
  /* Pilot reuse (Sec. 4.4), adaptive and chain frames: 1 = on the first frame
   * of each pilot pair (even frames; the second traces the same directions)
   * every probe's 8 pilot samples also update its caches, before the frame's
   * own samples, in octant order: each pilot's radiance into the irradiance
   * texel of its direction and its distance into the depth texel of its
   * direction. ADGI_FP32 / ADGI_FP16 storage, the per-sample wave blend. */
  int32_t pilot_reuse;
} adgi_update_params;

typedef struct {
  int64_t primary_rays;       /* rays traced from probes this frame               */
  int64_t pilot_rays;         /* 8 * P in adaptive mode                            */
  int64_t shadow_rays;        /* shadow rays of primary + pilot hits               */
  int64_t budget_used;        /* sum of rays per probe                             */
  uint32_t lambda;            /* allocation multiplier lambda*                      */
  int32_t n_min_seen, n_max_seen;
  float ms_total;             /* device time of the frame (sync = 1)               */
  float ms_stage[8];          /* eager launches with sync = 1: frame setup, pilot
                                 trace, detection, allocation, probe trace, blend,
                                 then the probe trace's two parts: closest-hit
                                 kernel and shading (shadow-ray) kernel (ms
                                 each); zero when the frame ran as a graph        */
  int64_t ties[4];            /* reserved                                          */
} adgi_update_stats;

/* Readback destinations (host). NULL fields are skipped. Texel arrays are
 * FP32 whatever the storage (FP16 is widened exactly, packed words decoded
 * on the host); with ADGI_PACKED the counts come from the words and the raw
 * words are available too. Debug arrays need ADGI_DEBUG_ARRAYS and hold the
 * last frame. */
typedef struct {
  float* irradiance;          /* [P][irr_res][irr_res][3]                          */
  float* depth;               /* [P][depth_res][depth_res][2] (tau, tau^2)         */
  uint8_t* irr_count;         /* [P][irr_res-2][irr_res-2] samples, saturating 255 */
  uint8_t* depth_count;       /* [P][depth_res-2][depth_res-2]                      */
  int32_t* rays_per_probe;    /* [P] n_i of the last frame                          */
  int64_t* score;             /* [P] detection score                                */
  int64_t* ray_offsets;       /* [P+1] exclusive prefix sum of rays_per_probe       */
  /* debug: per primary ray r = ray_offsets[i] + j of the last frame */
  int32_t* hit_tri;           /* [R] closest triangle, -1 for a miss               */
  uint8_t* shadow_bits;       /* [R] bit l: light l lit the hit point              */
  uint16_t* irr_bin;          /* [R] interior irradiance texel (row*(res-2)+col)   */
  uint16_t* depth_bin;        /* [R] interior depth texel                           */
  float* ray_record;          /* [R][4] radiance RGB, hit distance (inf = miss)    */
  uint16_t* q10_vis;          /* [P][8] pilot visibility code of the last frame    */
  uint16_t* q10_rad;          /* [P][8] pilot radiance code of the last frame      */
  float* frame_rotation;      /* [9] row-major rotation of the last frame          */
  int64_t num_rays;           /* out: R of the last frame                           */
  uint32_t* irr_words;        /* ADGI_PACKED: [P][irr_res][irr_res] raw words      */
  uint32_t* depth_words;      /* ADGI_PACKED: [P][depth_res][depth_res] raw words  */
  /* chain frames (max_chains > 0): after the last chain frame. With a chain
   * frame last, rays_per_probe / ray_offsets count samples per probe, the
   * per-ray debug arrays hold 2 * num_samples rays (sample k: rays 2k, 2k+1) */
  float* chain_state;         /* [chain_count][5] (p.xyz, u, v)                    */
  uint32_t* sample_probe;     /* [num_samples] probe of each sample, grouped       */
  float* sample_uv;           /* [num_samples][2] uv of each sample, grouped       */
  uint8_t* chain_accept;      /* debug: [chain_count][chain_steps] 1 = accepted    */
  int64_t num_samples;        /* out                                               */
  int32_t num_chains;         /* out: chain_count of the last chain frame (0: none) */
  int32_t chain_steps;        /* out: chain_steps of the last chain frame          */
  /* dynamic chains, after the last chain frame (max_chains > 0); with a chain
   * frame last, the debug arrays then hold 2 num_samples + num_dyn_rays rays */
  uint8_t* dyn_mark;          /* [Pp][8] marked (proxy, octant) of the last frame */
  float* dyn_target;          /* [Pp][8] F as the chains saw it (FP32)            */
  float* dyn_state;           /* [dyn_chain_count][5]                              */
  int64_t* dyn_ray_offsets;   /* [P+1] dynamic rays per probe, exclusive scan      */
  uint8_t* dyn_accept;        /* debug: [dyn_chain_count][dyn_chain_steps]         */
  int64_t num_dyn_rays;       /* out (0 without dynamic chains)                    */
  int32_t num_dyn_chains;     /* out: dyn_chain_count of the last chain frame      */
  int32_t dyn_chain_steps;    /* out                                               */
  int32_t proxy_dims[3];      /* out: ceil(dims / 3)                               */
  int32_t reserved;
  /* debug: the pilot rays of the last adaptive or chain frame, ray 8i + k */
  float* pilot_record;        /* [P][8][4] radiance RGB, hit distance (inf = miss);
                                 written on frames that reuse the pilots           */
  int32_t* pilot_tri;         /* [P][8] closest triangle, -1 for a miss            */
  uint8_t* pilot_shadow;      /* [P][8] bit l: light l lit the hit point           */
  uint16_t* pilot_ibin;       /* [P][8] interior irradiance texel (reuse frames)   */
  uint16_t* pilot_dbin;       /* [P][8] interior depth texel (reuse frames)        */
} adgi_probe_readback;

/* Create a volume: the uniform probe grid of Sec. 3.1 (probe i at origin +
 * (x, y, z) * spacing) with one octahedral irradiance tile and one
 * depth-moment (visibility) tile per probe, of the sizes of Tab.
 * probeDetails (8x8 and 16x16 with border by default). desc/alloc are host,
 * copied. hip_stream (hipStream_t or NULL) is the caller's stream: every call
 * orders its device work after the work already on that stream and makes
 * that stream wait for it. Texels and counts start at zero. *out receives the
 * handle, owned by the caller until adgi_destroy_volume. Errors:
 * ADGI_ERR_INVALID_ARG for a descriptor out of range (nothing allocated),
 * ADGI_ERR_OUT_OF_MEMORY when the allocator returns NULL (everything
 * allocated so far is released), ADGI_ERR_DEVICE when a HIP call fails. */
adgi_status adgi_create_volume(const adgi_volume_desc* desc, const adgi_allocator* alloc,
                               void* hip_stream, adgi_volume** out);

/* Upload or change the scene the probes see (Sec. 4.4 and 5: dynamic
 * lights and moving geometry between frames): triangles, per-triangle
 * albedo, point lights and sky. REBUILD builds a binned-SAH BVH on the host
 * and uploads it; REFIT uploads the changed vertex range and refits the
 * boxes on the device. Lights and sky are taken on every call. Asynchronous
 * w.r.t. the device; the host arrays are copied and may be reused on return.
 * Errors: ADGI_ERR_INVALID_ARG (NULL or non-finite arrays, indices out of
 * range, unknown mode), ADGI_ERR_NO_SCENE (REFIT before any REBUILD),
 * ADGI_ERR_TOPOLOGY (REFIT with another vertex or triangle count),
 * ADGI_ERR_OUT_OF_MEMORY, ADGI_ERR_DEVICE; on error the previous scene stays. */
adgi_status adgi_update_scene(adgi_volume* vol, const adgi_scene_desc* scene);

/* One probe-update frame, enqueued as one HIP graph launch: pilot rays and
 * change detection (Sec. 4.1, eq. ProbeVis, eq. priorDynamic), the split of
 * the frame's fixed sample budget over the probes (Sec. 3.3), ray tracing
 * with direct light at the hits (Sec. 3.1, 4.8), and the per-sample update of
 * the texel each sample falls in (Alg. ApproxAlgo, Alg. MovingAvgUpdate,
 * Sec. 4.5-4.7). params and stats are host memory; stats may be NULL and is
 * filled only when params->sync is 1 (the call then waits for the frame).
 * Errors (nothing enqueued): ADGI_ERR_NO_SCENE, ADGI_ERR_BUDGET,
 * ADGI_ERR_INVALID_ARG; ADGI_ERR_DEVICE when a HIP call fails (sticky). */
adgi_status adgi_update_probes(adgi_volume* vol, const adgi_update_params* params,
                               adgi_update_stats* stats);

/* For callers that cannot allocate device memory while frames run (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same frame as adgi_update_probes, same arguments and
 * results, bit for bit, but launched eagerly (no graph is instantiated) and
 * with the frame scratch taken from one fixed device array of
 * ADGI_STATIC_SCRATCH_BYTES per GPU, held from the first such call on that
 * GPU until the process ends. The call allocates nothing; the volume's own
 * state, records and debug arrays stay where adgi_create_volume put them.
 * Budgeted and uniform frames only. Every call on one GPU shares that GPU's
 * array and leaves its contents behind; the library orders these calls on
 * the GPU one after another (each waits for the previous call's frame), so
 * calls on different volumes and streams of one GPU do not overlap, which
 * they must not: two frames in the array at once would race.
 * Errors: those of adgi_update_probes; ADGI_ERR_INVALID_ARG for chain frames;
 * ADGI_ERR_BUDGET when the frame's scratch (about 60 bytes per hit slot,
 * max(B, 8 P) budgeted or P n_uniform uniform, plus about 140 bytes per probe)
 * exceeds ADGI_STATIC_SCRATCH_BYTES. */
#define ADGI_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
adgi_status adgi_update_probes_static(adgi_volume* vol, const adgi_update_params* params,
                                      adgi_update_stats* stats);

/* Wait for the volume's work and copy its probes into caller buffers: the
 * octahedral irradiance and depth-moment tiles a renderer reads at shading
 * points (Sec. 3.1's lookup; adgi_query_irradiance does that lookup on the
 * device), their sample counts, and the last frame's allocation and debug
 * arrays. out and every non-NULL field are host memory of the sizes given in
 * adgi_probe_readback. Errors: ADGI_ERR_INVALID_ARG (debug arrays without
 * ADGI_DEBUG_ARRAYS, raw words without ADGI_PACKED), ADGI_ERR_DEVICE. */
adgi_status adgi_read_probes(adgi_volume* vol, adgi_probe_readback* out);

/* Irradiance at shading points (the deferred-shading lookup of Sec. 3.1, with
 * DDGI's weights): the 8 probes of the grid cell around x (clamped to the
 * grid; an axis with one probe uses its one layer), each weighted by its
 * trilinear weight x (((dir.n + 1)/2)^2 + 0.2) (dir: unit vector from x to the
 * probe, n the unit normal) x (var / (var + (r - m)^2))^3 when
 * r = |x - p|/s exceeds the mean m of the probe's depth moments (m, m2) read
 * towards x (var = |m2 - m^2|), the product floored at 1e-6 before the
 * trilinear factor; out = the weighted mean of the probes' irradiance read
 * in direction n. Texels are read bilinearly across the tiles' borders.
 * points, normals, out_rgb: device memory, [count][3] FP32, owned by the
 * caller and not retained. Enqueued after the volume's frames (and the
 * caller's stream work); asynchronous like a frame. ADGI_FP32 and ADGI_FP16
 * storage (ADGI_ERR_INVALID_ARG for ADGI_PACKED). */
adgi_status adgi_query_irradiance(adgi_volume* vol, const float* points, const float* normals, int64_t count,
                                  float* out_rgb);

/* Complete pending work and release every device allocation. NULL is a no-op. */
void adgi_destroy_volume(adgi_volume* vol);

/* Message of the last failing call on this thread ("" if none). */
const char* adgi_last_error(void);

/* ---- launch tuning -------------------------------------------------------
 * How the frame is launched; results are bitwise identical for every valid
 * setting. Defaults: graph on, persistent traversal, autotuned sizes. */
typedef struct {
  int32_t use_graph;          /* 1: capture the frame as a hipGraph; 0: eager     */
  int32_t persistent;         /* 1: persistent traversal, a fixed grid whose waves
                                 take ray batches by grid stride (no shared
                                 counter): 64 rays, fewer in a pilot pass too
                                 small to fill the grid; 0: one thread per ray,
                                 grid sized to the rays                           */
  int32_t trace_block;        /* threads per traversal workgroup: 64..1024, x64
                                 (the fused pilot kernel runs the same number of
                                 waves, one per workgroup)                        */
  int32_t trace_waves_per_cu; /* persistent grid = CUs * this / (block/64), 1..32 */
  int32_t blend_chunk;        /* 0: wave-per-probe blend (tiles 8/16 or 16/16),
                                 probes taken in most-rays-first order;
                                 64..2048, x64: rays staged in LDS per step of the
                                 workgroup-per-probe blend                        */
  int32_t blend_blocks_per_cu;/* wave-per-probe blend: workgroups per CU, 1..32    */
  int32_t bvh_width;          /* 4: traverse the 4-wide BVH collapsed from the
                                 binary one (when its stack bound fits), else 2;
                                 2: the binary BVH                                */
  int32_t chain_lanes;        /* chain frames: 1 = one thread per chain, steps in
                                 sequence; 4 / 8 / 16 / 32 = prefetching groups of
                                 that many lanes per chain, 2..5 steps per round
                                 (Brockwell 2006), the same chains bit for bit;
                                 0 = chosen from the chain count                  */
  int32_t ray_order;          /* probe rays: 1 = each wave traces a compact patch
                                 of directions (a probe's spherical Fibonacci
                                 indices cut into bands, each band taken in
                                 azimuth order); 0 = index order                  */
} adgi_tuning;

/* ---- packed texel channels (eq. rgbEnc, App. B) ---------------------------
 * Round trip of `count` binary32 values through one channel of the packed
 * 32-bit texels, with the encoder and decode tables of the packed blend:
 * codes[i] = floor(qmax min(ln(gamma x + 1), beta) / beta) (qmax = 2^bits - 1,
 * the exact floor; x < 0 counts as 0) and decoded[i] = (e^(beta code / qmax)
 * - 1) / gamma rounded to binary32. Channels: ADGI_PACK_RG9 (irradiance R and
 * G, 9 bits, beta 5, gamma 15), ADGI_PACK_B8 (B, 8 bits, 5, 15),
 * ADGI_PACK_TAU13 (mean distance, 13 bits, 5, 15), ADGI_PACK_TAU2_13 (mean
 * squared distance, 13 bits, 8, 20). values, codes, decoded: device memory
 * of `count` elements, owned by the caller; codes or decoded may be NULL.
 * Enqueued on hip_stream (NULL: the default stream) on the current device,
 * asynchronous; the first call on a device uploads the tables (68.6 KB,
 * kept for the process). Errors: ADGI_ERR_INVALID_ARG (count < 0, unknown
 * channel, NULL arrays), ADGI_ERR_DEVICE. */
enum { ADGI_PACK_RG9 = 0, ADGI_PACK_B8 = 1, ADGI_PACK_TAU13 = 2, ADGI_PACK_TAU2_13 = 3 };
adgi_status adgi_pack_channel(const float* values, int64_t count, int32_t channel, uint32_t* codes,
                              float* decoded, void* hip_stream);

adgi_status adgi_get_tuning(const adgi_volume* vol, adgi_tuning* out);
adgi_status adgi_set_tuning(adgi_volume* vol, const adgi_tuning* t);
/* Time candidate launch shapes on the current scene and frame parameters
 * and keep the fastest. Runs one frame, then the traversal and the blend
 * several times each, in place, and restores the volume's state from a
 * snapshot taken first: the state afterwards is bit-identical. The choice is
 * cached per (device, shape class) in memory for the process. */
adgi_status adgi_autotune(adgi_volume* vol, const adgi_update_params* params, adgi_tuning* chosen);

/* ---- traversal work (for rooflines) --------------------------------------
 * Runs the frame's pilot/detection/allocation steps and a counting variant of
 * the probe-ray traversal (same rays, same kernel shape) on the current
 * scene, then restores the volume's state. node_tests counts node visits
 * (a BVH2 visit tests two child boxes, a BVH4 visit four), tri_tests
 * ray/triangle tests, both over the probe rays and their shadow rays;
 * shade_node_tests and shade_tri_tests are the shadow rays' share (the
 * shading kernel's work). */
typedef struct {
  int64_t primary_rays, shadow_rays, node_tests, tri_tests;
  int64_t box_tests;          /* child boxes tested: 2 per BVH2 visit, the
                                 non-empty child slots of a BVH4 visit       */
  int64_t shade_node_tests, shade_tri_tests;
  int64_t shade_box_tests;    /* the shading kernel's part of box_tests      */
} adgi_trace_work;
adgi_status adgi_measure_trace_work(adgi_volume* vol, const adgi_update_params* params,
                                    adgi_trace_work* out);

/* ---- state snapshot (checkpoint / eviction) ------------------------------
 * The complete temporal state: texels, counts, detection codes and triggers,
 * scores and the last frame's allocation. Restoring a snapshot into a volume
 * created with the same desc resumes bit-identically. */
size_t adgi_state_size(const adgi_volume* vol);
adgi_status adgi_save_state(adgi_volume* vol, void* host_dst, size_t bytes);
adgi_status adgi_restore_state(adgi_volume* vol, const void* host_src, size_t bytes);
/* Device bytes the volume holds now (state + scene + frame buffers). */
size_t adgi_device_bytes(const adgi_volume* vol);

/* ---- serving: many volumes on one GPU -------------------------------------
 * A server holds streams; each stream is one probe volume with its own scene,
 * grid, budget and frame parameters (adaptive frames only). A request asks
 * for the stream's next frame with that frame's light positions. Requests are
 * dispatched in arrival order, at most one frame of a stream and at most
 * max_inflight frames in total at a time, on min(2 max_inflight, 16)
 * streams the server creates ("lanes"; an idle volume takes the next
 * least-loaded lane in rotation for its next frame). Resident streams are served first. HBM admission: a stream's volume is
 * resident only while the device bytes of all resident volumes stay within
 * hbm_budget_bytes; to admit one, idle resident streams with nothing waiting
 * are evicted, least recently used first (a request waiting over 250 ms may
 * also evict idle streams resident for over 500 ms). Eviction enqueues the
 * copy of the temporal state to pinned host memory and frees all the
 * volume's device memory once it has landed (until then the bytes stay
 * counted against the budget); re-admission rebuilds the volume from the BVH
 * the server built once per stream (uploaded from a pinned copy) and
 * restores the state, and its first frame is dispatched once those copies
 * have landed, so a stream's results are bitwise those it would have alone. The server is not thread-safe; its
 * own errors are described by adgi_server_last_error (volume errors by
 * adgi_last_error). The scene arrays of adgi_server_add_stream are copied. */
typedef struct adgi_server adgi_server;
typedef struct {
  int64_t hbm_budget_bytes;   /* > 0: device bytes of resident volumes, at most */
  int32_t max_inflight;       /* 1..64: frames in flight across all streams      */
  int32_t reserved;
} adgi_server_desc;
typedef struct {
  adgi_volume_desc volume;
  adgi_scene_desc scene;      /* REBUILD description; light_pos = initial lights */
  adgi_update_params params;  /* adaptive = 1; frame and sync are set per request */
} adgi_stream_desc;
typedef struct {
  int64_t submitted, completed, admissions, evictions;
  int64_t primary_rays;       /* budget of every completed frame                  */
  int64_t resident_bytes, peak_resident_bytes;
  double p50_ms, p99_ms, mean_ms, max_ms;  /* arrival -> frame seen done (event) */
  double span_s;              /* first arrival -> last completion                 */
  double admit_ms, evict_ms;  /* host time spent admitting and evicting          */
  double device_busy_ms;      /* sum over completed frames of their device span
                                 (an event on the lane before the frame's scene
                                 update to one after its blend): divided by the
                                 wall time it is the mean number of frames on
                                 the device at once                              */
} adgi_server_stats;

int64_t adgi_server_now_ns(void);  /* steady clock used for arrival stamps        */
const char* adgi_server_last_error(void);
adgi_status adgi_server_create(const adgi_server_desc* desc, const adgi_allocator* alloc, adgi_server** out);
/* Builds the stream's BVH on the host and measures its device footprint with
 * one dry frame; the stream starts evicted with zero state at frame 0.
 * ADGI_ERR_OUT_OF_MEMORY if the footprint alone exceeds the budget. */
adgi_status adgi_server_add_stream(adgi_server* s, const adgi_stream_desc* d, int32_t* stream_id);
adgi_status adgi_server_set_budget(adgi_server* s, int64_t hbm_budget_bytes);
adgi_status adgi_server_stream_info(const adgi_server* s, int32_t stream_id, int64_t* footprint_bytes,
                                    int32_t* resident, int32_t* frames_done);
/* light_pos: [num_lights][3] for this frame (copied); arrival_ns on the
 * adgi_server_now_ns clock (latency is measured from it). */
adgi_status adgi_server_submit(adgi_server* s, int32_t stream_id, const float* light_pos, int64_t arrival_ns);
/* Non-blocking: retires finished frames, admits/evicts, dispatches. */
adgi_status adgi_server_progress(adgi_server* s, int32_t* completed_now);
/* Blocks until every submitted request is done. */
adgi_status adgi_server_drain(adgi_server* s);
adgi_status adgi_server_get_stats(const adgi_server* s, adgi_server_stats* out);
/* Per-request latencies (ms) in completion order; count = all recorded. */
adgi_status adgi_server_latencies(const adgi_server* s, double* out_ms, int64_t capacity, int64_t* count);
/* Readback of an idle stream (admitted first if evicted). */
adgi_status adgi_server_read_stream(adgi_server* s, int32_t stream_id, adgi_probe_readback* rb);
void adgi_server_destroy(adgi_server* s);

#ifdef __cplusplus
}
#endif
#endif
