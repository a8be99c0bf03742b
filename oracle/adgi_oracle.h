/* adgi_oracle.h - FP64 CPU oracle for the adaptive probe-update path.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or constant generator with the GPU library; the two are
 * written independently from the paper and meet only on the seeded inputs.
 *
 * The oracle is the method's steps written out plainly in double precision:
 *   - octahedral direction map and its border fold,
 *   - counter-based random numbers, per-frame rotation, spherical Fibonacci
 *     ray sets and octant-stratified pilot directions,
 *   - closest-hit and any-hit queries (Moller-Trumbore, brute force or a
 *     median-split BVH of its own),
 *   - direct-light shading with shadow rays,
 *   - change detection (probe visibility f_v = exp(-2t/s), eq. ProbeVis;
 *     incoming radiance f_r = min(r, beta)/beta, Sec. 4.1.3; temporal
 *     gradients, eq. tempGradVis / tempGradIrr; temporal trigger and 5x5x5
 *     spatial sum, Sec. 4.1.4-4.1.5; dynamic composition, eq. priorDynamic),
 *   - integer ray-budget allocation,
 *   - the per-sample moving average of Alg. MovingAvgUpdate applied to the
 *     texel containing each sample (Alg. ApproxAlgo).
 *
 * Ties: where FP32 (GPU) and FP64 (oracle) arithmetic can legitimately take
 * different discrete decisions (which triangle is hit, whether a shadow ray
 * is blocked, which texel a direction falls in, which 10-bit code a value
 * quantises to), the oracle flags the decision as a tie. Callers may pass
 * the GPU's decisions as hints; on a tie the oracle adopts the hint and
 * counts it, and a differing hint that is not a tie counts as a mismatch.
 */
#ifndef ADGI_ORACLE_H
#define ADGI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers (splitmix64, Steele, Lea & Flood 2014) */
uint64_t orc_splitmix64(uint64_t x);
uint64_t orc_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c);
double   orc_uniform(uint64_t key, uint64_t q);   /* top 24 bits of mix(key^q) * 2^-24 */
#define ORC_TAG_ROTATION 0x524F54ull  /* "ROT" */
#define ORC_TAG_PILOT    0x50494Cull  /* "PIL" */
#define ORC_TAG_CHAIN    0x4D4353ull  /* "MCS": a Metropolis step */
#define ORC_TAG_CHAININIT 0x4D4349ull /* "MCI": a chain's first state */
#define ORC_TAG_DYNCHAIN 0x4D4453ull  /* "MDS": a dynamic-chain step */
#define ORC_TAG_DYNCHAININIT 0x4D4449ull /* "MDI": a dynamic chain's first state */

/* Per-frame rotation (Shoemake, Graphics Gems III 1992), FP64 -> FP32. */
void orc_frame_rotation(uint64_t seed, int32_t frame, float R[9]);
/* Spherical Fibonacci direction j of n, rotated by R (FP64). */
void orc_sf_dir(int32_t j, int32_t n, const float R[9], double d[3]);
/* Spherical Fibonacci point (index) that ray j of a probe with n rays takes. */
int32_t orc_ray_point(int32_t j, int32_t n);
/* Pilot direction: probe, octant k (bit0 -x, bit1 -y, bit2 -z), pair m. */
void orc_pilot_dir(uint64_t seed, int32_t probe, int32_t k, int32_t pair, double d[3]);

/* ---- octahedral map (Cigolle et al. 2014) */
void orc_oct_encode(const double d[3], double uv[2]);
void orc_oct_decode(const double uv[2], double d[3]);
/* interior bin k = iy*r + ix; *tie set when a cell edge is within eps */
int32_t orc_oct_bin(const double d[3], int32_t r, double eps, int32_t* tie);
/* source interior coordinate (1..r) of tile coordinate (X,Y) in 0..r+1 */
void orc_border_source(int32_t X, int32_t Y, int32_t r, int32_t* sx, int32_t* sy);
/* interior [r*r*c] -> full tile [(r+2)*(r+2)*c] with border fold */
void orc_fold_tile(const double* interior, int32_t r, int32_t c, double* tile);

/* ---- tolerances that define ties */
typedef struct {
  double hit_rel;     /* another surface within hit_rel*t of the closest hit   */
  double edge_rel;    /* world margin = edge_abs + edge_rel*(|o|_inf + t + |v|) */
  double edge_abs;
  double graze;       /* |cos(ray, plane normal)| below this is a tie          */
  double bin_eps;     /* bin coordinate within bin_eps of a cell edge          */
  double q10_rel;     /* code coordinate within q10_abs + q10_rel*x*1024 ...   */
  double q10_abs;
  double cos_eps;     /* light cosine within cos_eps of 0                       */
} orc_tol;
void orc_default_tol(orc_tol* tol);

/* ---- scene */
typedef struct orc_scene orc_scene;
orc_scene* orc_scene_new(int32_t nv, const float* pos, int32_t nt, const int32_t* idx,
                         const float* albedo, int32_t use_bvh);
void orc_scene_free(orc_scene* s);
void orc_scene_set_positions(orc_scene* s, const float* pos);  /* rebuilds the BVH */
void orc_scene_set_lights(orc_scene* s, int32_t nl, const float* lpos, const float* lint,
                          const float sky[3]);
int32_t orc_scene_bvh_depth(const orc_scene* s);

typedef struct {
  double t;        /* hit distance, INFINITY on a miss */
  int32_t tri;     /* -1 on a miss */
  int32_t front;   /* 1 if (v1-v0)x(v2-v0) . d < 0 */
  int32_t tie;     /* decision is within the tie tolerance */
} orc_hit;

/* exact closest hit: brute force over all triangles, or the oracle's BVH */
void orc_closest_hit(const orc_scene* s, const double o[3], const double d[3],
                     const orc_tol* tol, orc_hit* out);
void orc_closest_hit_brute(const orc_scene* s, const double o[3], const double d[3],
                           const orc_tol* tol, orc_hit* out);
/* any hit on (0, tmax); *tie set when ambiguous */
int32_t orc_occluded(const orc_scene* s, const double o[3], const double d[3], double tmax,
                     const orc_tol* tol, int32_t* tie);

/* ---- one probe ray: trace + shade (O3, O4) */
typedef struct {
  double rgb[3];
  double t;
  int32_t tri;
  int32_t front;
  uint8_t shadow;       /* bit l: light l lit the hit point (cos > 0 and unblocked) */
  int32_t hit_tie, shadow_tie;
} orc_ray;
/* hint_tri: GPU hit triangle or -2 for none; hint_shadow: GPU light bits */
void orc_shade_ray(const orc_scene* s, const double o[3], const double d[3], double spacing_diag,
                   const orc_tol* tol, int32_t hint_tri, int32_t hint_shadow, orc_ray* out,
                   int64_t* ties, int64_t* mismatches);

typedef struct {
  int64_t hit_ties, shadow_ties, bin_ties, q10_ties;
  int64_t hit_mismatch, shadow_mismatch, bin_mismatch, q10_mismatch;
  int64_t rays, shadow_rays;
  int64_t chain_ties, chain_mismatch;  /* Metropolis accept decisions */
} orc_counts;

/* ---- grid */
typedef struct {
  double origin[3], spacing[3];
  int32_t dims[3];
  double s;            /* ||spacing||_2 : voxel (cage) diagonal */
} orc_grid;
void orc_grid_init(orc_grid* g, const float origin[3], const float spacing[3], const int32_t dims[3]);
void orc_probe_pos(const orc_grid* g, int32_t i, double p[3]);

/* ---- detection (O5): pilots for every probe, Q10 codes with ties.
 * hint_qv/hint_qr may be NULL; otherwise tied codes adopt the hint.
 * hint_tri/hint_shadow [P*8] may be NULL; otherwise the pilot rays adopt the
 * tied hit and shadow decisions (as probe rays do). prgb [P*8*3] and pt
 * [P*8], if not NULL, receive each pilot's radiance and hit distance. */
void orc_pilots(const orc_scene* s, const orc_grid* g, uint64_t seed, int32_t frame,
                double beta, const orc_tol* tol, const uint16_t* hint_qv, const uint16_t* hint_qr,
                const int32_t* hint_tri, const uint8_t* hint_shadow,
                uint16_t* qv, uint16_t* qr, double* prgb, double* pt, orc_counts* counts);
/* ---- pilot reuse (Sec. 4.4): the 8 pilot samples of each listed probe
 * update its caches like probe rays, in octant order: pilot k's radiance
 * (prgb, from orc_pilots) into the irradiance texel of its direction, its
 * distance (pt) into the depth texel of its direction. State arrays are
 * indexed by position in the list as for orc_probes_frame; hint_ibin /
 * hint_dbin [P*8] may be NULL. */
void orc_pilot_blend(const orc_grid* g, uint64_t seed, int32_t frame, int32_t count, const int32_t* probes,
                     const orc_tol* tol, int32_t irr_r, int32_t dep_r, double hysteresis, double tau_max,
                     const double* prgb, const double* pt, const uint16_t* hint_ibin,
                     const uint16_t* hint_dbin, double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                     orc_counts* counts);
/* state arrays are [P*8]; score is [P]. Updates the state for frame t. */
void orc_detect(const orc_grid* g, int32_t frame, int32_t theta, int32_t mu,
                const uint16_t* qv, const uint16_t* qr, uint16_t* qv_prev, uint16_t* qr_prev,
                int32_t* tv, int32_t* tr, int64_t* score);

/* ---- allocation (O6). Returns 0 or -1 (budget below P*n_min). */
int32_t orc_allocate(int32_t P, const int64_t* score, int64_t budget, int32_t n_min, int32_t n_max,
                     int32_t* n, int64_t* offsets, uint32_t* lambda_out);

/* ---- one probe's frame: trace its n rays, blend them (O2-O4, O7).
 * irr[36*3], irr_n[36], dep[196*2], dep_n[196] are the interior state in
 * FP64 (updated in place). Optional hints are indexed by ray j. Optional
 * outputs: rays[n*4] (rgb, t), tri[n], shadow[n], ibin[n], dbin[n]. */
void orc_probe_frame(const orc_scene* s, const orc_grid* g, int32_t probe, int32_t n,
                     const float R[9], const orc_tol* tol,
                     int32_t irr_r, int32_t dep_r, double hysteresis, double tau_max, int32_t fp16,
                     const int32_t* hint_tri, const uint8_t* hint_shadow,
                     const uint16_t* hint_ibin, const uint16_t* hint_dbin,
                     double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                     double* rays, int32_t* tri, uint8_t* shadow, uint16_t* ibin, uint16_t* dbin,
                     orc_counts* counts);
/* many probes in parallel (OpenMP); state arrays indexed by position in list;
 * hints/outputs indexed by ray offset ray_base[q] + j. gather != 0 replaces the
 * per-sample update by DDGI's gather (Majercik et al. 2019, the blend Sec. 3.1
 * describes): every texel takes the frame's rays weighted by max(0, c.d) (c
 * its centre direction; depth: that cosine to the 50th power), and the
 * weighted mean enters the texel with a = max(1/(N+1), 1-h), N counting the
 * frames in which the texel had weight. */
void orc_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                      const int32_t* n, const int64_t* ray_base, const float R[9], const orc_tol* tol,
                      int32_t irr_r, int32_t dep_r, double hysteresis, double tau_max, int32_t fp16,
                      int32_t gather, const int32_t* hint_tri, const uint8_t* hint_shadow,
                      const uint16_t* hint_ibin, const uint16_t* hint_dbin,
                      double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                      double* rays, int32_t* tri, uint8_t* shadow, uint16_t* ibin, uint16_t* dbin,
                      orc_counts* counts);

/* single moving-average step of Alg. MovingAvgUpdate with real N_max */
double orc_blend_alpha(int32_t n, double hysteresis);
/* binary16 round-to-nearest-even of a double */
double orc_round_half(double x);

/* ---- packed 32-bit texels (eq. rgbEnc; Sec. 4.6; App. B) ----------------
 * The texel values are binary32 (the paper's shader arithmetic: the moving
 * average runs in binary32, fused multiply-adds explicit); the codes are the
 * exact eq. rgbEnc of those binary32 values and the decoded values the exact
 * ones rounded once to binary32, both through FP64 libm. */
/* floor(min(ln(gamma v + 1), beta) / beta * (2^bits - 1)) for v >= 0, exact */
uint32_t orc_pack_encode(float v, float beta, float gamma, int32_t bits);
/* (exp(beta q / (2^bits - 1)) - 1) / gamma, rounded to binary32 */
float orc_pack_decode(uint32_t q, float beta, float gamma, int32_t bits);
/* Moving average of Alg. MovingAvgUpdate on packed words, samples of each
 * probe applied in ray order: irradiance word = R9 | G9 << 9 | B8 << 18 |
 * N6 << 26 (beta 5, gamma 15), depth word = tau13 | tau^2_13 << 13 | N6 << 26
 * (beta 5 / gamma 15 and beta 8 / gamma 20). rec[r] = (R, G, B, t) as the
 * trace wrote it (FP32); tau = min(t * inv_s, tau_max); alpha[N] the step
 * weight for count N (N saturates at 63). irr: [count][ri*ri], dep:
 * [count][rd*rd] interior words, updated in place. */
void orc_packed_blend(int32_t count, const int32_t* n, const int64_t* ray_base, const float* rec,
                      const uint16_t* ibin, const uint16_t* dbin, int32_t ri, int32_t rd, float inv_s,
                      float tau_max, const float* alpha, uint32_t* irr, uint32_t* dep);

/* ---- Metropolis chains over (position, direction) (Sec. 3.2-3.3, Alg.
 * MarkovChainMT, Alg. MetropolisStep, Sec. 4.8: the static chain).
 * State x = (p, uv): p in the box spanned by the probe centres, uv the
 * octahedral coordinates of the direction in [-1, 1]^2. Target
 * h = exp(min(g/f, 1)) f, f = Qv/1024 of the nearest probe's octant of the
 * direction (the 10-bit f_v code of the current frame's pilots), g the
 * luminance of that probe's irradiance averaged over the 2x2 texels (one
 * level coarser) whose cell holds uv, from the previous frame; h = 0 where
 * f = 0. Step i of frame t for chain c draws u1..u7 from key (seed, MCS, c,
 * t, i): Box-Muller normals (u1,u2) -> g1,g2, (u3,u4) -> g3,g4, (u5,u6) -> g5,
 * proposal p' = p + sigma_pos*spacing*(g1,g2,g3), uv' = uv + sigma_dir*(g4,g5);
 * a proposal outside the domain is rejected; otherwise it is accepted when
 * the current density is 0 or u7*h(x) <= h(x'). Steps i > burn_in emit the
 * state after the step: S = steps - burn_in - 1 samples per chain and frame,
 * sample c*S + i - burn_in - 1, as (nearest probe, uv). */
typedef struct {
  int32_t chains, steps, burn_in;
  double sigma_pos, sigma_dir;
} orc_chain_params;
/* probe: nearest probe; tie: the evaluation sits within tolerance of a
 * discrete boundary (domain, nearest probe, octant, coarse cell). */
double orc_chain_h(const orc_grid* g, const uint16_t* qv, const double* irr_prev, int32_t r,
                   const double x[5], int32_t* probe, int32_t* tie);
/* One frame of every chain. state [C][5] (p, uv) in/out; init != 0 draws the
 * first states from key (seed, MCI, c, 0, 0) (p uniform in the box, uv
 * uniform in the square). irr_prev: interior irradiance [P][r*r][3].
 * hint_accept [C][steps] (optional): the GPU's decisions, adopted where the
 * oracle's decision is a tie (counted) and counted as mismatches elsewhere.
 * Outputs (optional): accept [C][steps], sample_probe [C*S], sample_uv [C*S][2]. */
void orc_chain_frame(const orc_grid* g, const orc_chain_params* cp, uint64_t seed, int32_t frame,
                     const uint16_t* qv, const double* irr_prev, int32_t r, double* state, int32_t init,
                     const uint8_t* hint_accept, uint8_t* accept, int32_t* sample_probe,
                     double* sample_uv, orc_counts* counts);
/* Octahedral decode of uv to a unit direction (O1). */
void orc_chain_dir(const double uv[2], double d[3]);
/* Chain samples of the listed probes, each probe's samples in ascending
 * sample order: ray along d(uv) from the probe centre (shaded, as probe rays)
 * updates the irradiance texel of d; ray along -d updates the depth texel of
 * -d with its distance (the visibility ray of Sec. 4.8). Samples of list
 * entry q: [sample_base[q], sample_base[q] + nsamp[q]) of sample_uv; hints
 * and ray outputs indexed 2k (ray along d) and 2k+1 (along -d). quant
 * (optional, per list entry): nonzero traces the two rays through the centres
 * of the irradiance texel of d and of the depth texel of -d instead. */
void orc_chain_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                            const int32_t* nsamp, const int64_t* sample_base, const double* sample_uv,
                            const uint8_t* quant, const orc_tol* tol, int32_t irr_r, int32_t dep_r, double hysteresis,
                            double tau_max, int32_t fp16, const int32_t* hint_tri, const uint8_t* hint_shadow,
                            const uint16_t* hint_ibin, const uint16_t* hint_dbin, double* irr,
                            uint8_t* irr_n, double* dep, uint8_t* dep_n, orc_counts* counts);

/* ---- dynamic chains on virtual proxies (Sec. 4.9) -----------------------
 * f_d of every (probe, octant), eq. priorDynamic with f_c = 1: Qv (Cv + mu Cr),
 * C the 5x5x5 sums (zero outside the grid) of the triggers Tv, Tr, Qv the
 * pilot visibility codes of the frame that last ran detection. */
void orc_dynamic_fd(const orc_grid* g, int32_t mu, const uint16_t* qv, const int32_t* tv, const int32_t* tr,
                    int64_t* fd);
/* Virtual proxies: groups of 3x3x3 probes (proxy (X,Y,Z) holds probes with
 * x/3 = X, y/3 = Y, z/3 = Z; the last group along an axis may be smaller),
 * proxy grid ceil(dims/3). F[proxy][octant] = max of f_d over its probes. */
void orc_proxy_dims(const orc_grid* g, int32_t pd[3]);
int32_t orc_proxy_of_probe(const orc_grid* g, int32_t probe);
void orc_proxy_max(const orc_grid* g, const int64_t* fd, int64_t* F);
/* One frame of the dynamic chains: the same random walk as the static chain
 * (keys MDS / MDI instead of MCS / MCI) on the target h = F[proxy of the
 * nearest probe][octant of uv] (alpha = 0). Every state past the burn-in with
 * h > 0 sets mark[proxy][octant] = 1 (each marked octant is updated once). */
void orc_dyn_chain_frame(const orc_grid* g, const orc_chain_params* cp, uint64_t seed, int32_t frame,
                         const int64_t* F, double* state, int32_t init, const uint8_t* hint_accept,
                         uint8_t* accept, uint8_t* mark, orc_counts* counts);
/* Interior texels (row-major y*r + x) whose centres lie in octant k, in
 * ascending order: centre uv = ((2x+1)/r - 1, (2y+1)/r - 1), octant bits
 * u < 0, v < 0, |u| + |v| > 1 (centres on the diagonal belong to the upper
 * half); returns the count; list may be NULL. */
int32_t orc_octant_texels(int32_t r, int32_t k, int32_t* list);
/* Unit direction through the centre of interior texel t of an r x r map. */
void orc_texel_centre_dir(int32_t r, int32_t t, double d[3]);
/* Dynamic rays of a probe whose proxy has the octants in octant_mask marked. */
int32_t orc_dyn_ray_count(int32_t irr_r, int32_t dep_r, uint32_t octant_mask);
/* Dynamic updates of the listed probes, after the frame's static samples: for
 * each marked octant of the probe's proxy, ascending, one shaded ray through
 * the centre of each irradiance texel of the octant (into that texel) and
 * then one ray through the centre of each depth texel of the octant (its
 * distance into that texel), both with a = max(1/(N+1), 1 - h_dyn). Ray j of
 * list entry q is hint index ray_base[q] + j. fp16: round the tiles to
 * binary16 at the end (the frame's only store). */
void orc_dyn_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                          const uint8_t* mark, const int64_t* ray_base, const orc_tol* tol, int32_t irr_r,
                          int32_t dep_r, double h_dyn, double tau_max, int32_t fp16, const int32_t* hint_tri,
                          const uint8_t* hint_shadow, double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                          orc_counts* counts);

/* ---- irradiance query (the deferred-shading lookup of Sec. 3.1, DDGI) -----
 * Irradiance at a point x with unit normal n from the 8 probes of the grid
 * cell around x (clamped to the grid; an axis with one probe uses one layer):
 * weight of a probe = trilinear weight x (((dir.n + 1)/2)^2 + 0.2) (dir from x
 * to the probe) x Chebyshev visibility (if r = |x - p|/s exceeds the mean tau
 * of the probe's depth moments towards x: (var / (var + (r - mean)^2))^3,
 * var = |mean2 - mean^2|), floored at 1e-6 before the trilinear factor; the
 * result is the weighted mean of the probes' irradiance in direction n.
 * Texels are read bilinearly from full tiles (with borders): irr_tiles
 * [P][irr_res][irr_res][3], dep_tiles [P][dep_res][dep_res][2]. */
void orc_query_irradiance(const orc_grid* g, const double* irr_tiles, int32_t irr_res, const double* dep_tiles,
                          int32_t dep_res, const double x[3], const double n[3], double rgb[3]);

int32_t orc_num_threads(void);
/* Threads for the following OpenMP regions (timing only). */
void orc_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
