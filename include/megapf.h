/*
 * megapf.h -- C-ABI of libmegapf, an MI355X (gfx950) implementation of the
 * correction hot path of the Gauss-Newton Stein particle filter of
 * Koide, Oishi, Yokozuka, Banno, "MegaParticles: Range-based 6-DoF Monte
 * Carlo Localization with GPU-Accelerated Stein Particle Filter", ICRA 2024.
 *
 * Problem (Sec. III-A): estimate the sensor pose T_t on a point-cloud map M
 * from a scan P_t with a set of SE(3) particles X_t = {T_t^i}.
 *
 * Conventions shared by every call
 *   - Status: 0 (MP_OK) or a negative MP_E_* code.  On error nothing the call
 *     would have produced is modified, and mp_last_error() returns a message
 *     for the calling thread.  A handle stays valid after an error.
 *   - Pointers: every array argument may be a host pointer or a device pointer
 *     of the current HIP device (unified addressing decides).  The library
 *     never keeps a caller pointer: data is copied in stream order before the
 *     call returns (host memory) or before the stream passes the copy (device
 *     memory).  Outputs written to host memory are complete when the call
 *     returns (the call synchronises the stream first).
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  From PyTorch on ROCm: torch.cuda.current_stream().cuda_stream.
 *     Every call is asynchronous on that stream except where host outputs are
 *     requested.
 *   - Units: metres and radians.  Poses are (qw, qx, qy, qz, tx, ty, tz):
 *     a Hamilton unit quaternion and a translation, mapping sensor-frame
 *     points into the map frame.  Tangent vectors are [omega; v] (rotation
 *     first, the order of the kernel weight W^K in Eq. 7) and perturb on the
 *     right: T exp(delta) (Eq. 1 and Eq. 5).
 *   - Handles are created and freed only by the library.  A map may serve
 *     several filters and must outlive them.
 */
#ifndef MEGAPF_H
#define MEGAPF_H

#include <stdint.h>

#if defined(__GNUC__)
#define MP_API __attribute__((visibility("default")))
#else
#define MP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mp_status;
enum {
    MP_OK = 0,
    MP_E_ARG = -1,         /* invalid argument (null, size, non-finite value) */
    MP_E_STATE = -2,       /* call not valid in the handle's current state */
    MP_E_OOM = -3,         /* device allocation failed */
    MP_E_HIP = -4,         /* HIP runtime error; the HIP message is in mp_last_error() */
    MP_E_UNSUPPORTED = -5, /* valid request outside the implemented limits */
    MP_E_NUMERIC = -6      /* a non-finite value appeared in the filter state */
};

typedef struct mp_map_s* mp_map;
typedef struct mp_filter_s* mp_filter;

/* ------------------------------------------------------------------ map */

enum { MP_NNF_AUTO = 0, MP_NNF_HASH = 1, MP_NNF_DENSE = 2 };

/* Map elements (Sec. III-C):
 *   VOXEL  one Gaussian per voxel holding >= min_points map points; the field
 *          maps each voxel within Chebyshev distance R of a kept voxel to the
 *          kept voxel at the smallest integer squared offset.
 *   POINT  the paper's construction: one Gaussian per map point, from the
 *          point and its point_k nearest other map points among those whose
 *          voxel lies within Chebyshev distance point_search (kept when that
 *          neighbourhood holds >= min_points points); the field, a grid of
 *          cell edge `voxel`, maps each cell to the kept point nearest to the
 *          cell's centre within nnf_radius * voxel (nnf_radius >= 1; DENSE
 *          backend only). */
enum { MP_GAUSS_VOXEL = 0, MP_GAUSS_POINT = 1 };

typedef struct {
    float voxel;        /* voxel edge r in metres, > 0 (POINT: the field's cell edge) */
    int32_t nnf_radius; /* Chebyshev radius of the nearest-neighbour band, voxels, 0..8 */
    int32_t min_points; /* voxels (POINT: neighbourhoods) holding fewer map points are dropped, >= 3 */
    float cov_eps;      /* GICP normalisation: Sigma = I - (1 - eps) n n^T, 0 < eps <= 1 */
    int32_t backend;    /* MP_NNF_*: open-addressing voxel hash map or dense grid;
                           AUTO picks DENSE when the band grid has <= 2^26 cells and
                           < 2^24 cells per z plane; DENSE beyond 2^27 - 2 cells or
                           2^24 per plane fails with MP_E_UNSUPPORTED */
    int32_t gauss_mode;   /* MP_GAUSS_*: map elements */
    int32_t point_k;      /* POINT: neighbours per point, 3..32 */
    int32_t point_search; /* POINT: Chebyshev voxel radius of the neighbour search, 1..4 */
} mp_map_params;

typedef struct {
    int64_t num_gauss;       /* occupied voxels kept (Gaussians) */
    int64_t num_band;        /* voxels of the nearest-neighbour band */
    int32_t grid_origin[3];  /* voxel coordinate of band-grid cell (0,0,0) */
    int32_t grid_dim[3];     /* band-grid extent in voxels */
    float box_min[3];        /* corners of the kept voxels, metres */
    float box_max[3];
    int32_t backend;         /* MP_NNF_HASH or MP_NNF_DENSE actually built */
    int64_t table_slots;     /* hash slots or dense cells */
    int64_t device_bytes;    /* device memory held by the map */
} mp_map_info;

/* Fill defaults: voxel 0.5, nnf_radius 2, min_points 5, cov_eps 1e-3, AUTO,
 * VOXEL Gaussians, point_k 10, point_search 2. */
MP_API void mp_map_default_params(mp_map_params* p);

/* Build the per-voxel Gaussian map and its nearest-neighbour field
 * (Sec. III-C "Likelihood evaluation": each map point is a Gaussian
 * N(mu, Sigma); m^nnf gives, for a voxel of space, the index of the nearest
 * map Gaussian).
 *   xyz   n x 3 float32 map points (host or device), row-major.
 *   Points are grouped by voxel v = floor(p * (1/r)) (FP32).  A voxel with at
 *   least min_points points yields one Gaussian: mean, and the GICP-normalised
 *   covariance I - (1-eps) n n^T where n is the eigenvector of the smallest
 *   eigenvalue of the 1/n sample covariance (Segal et al. 2009).  Gaussian ids
 *   follow ascending (vz, vy, vx).  Every voxel within Chebyshev distance R of
 *   a kept voxel maps to the kept voxel at the smallest integer squared
 *   distance, ties to the smaller id; other voxels are misses.
 * With gauss_mode POINT the Gaussians are the map points themselves (mu = p,
 * count = size of the neighbourhood) in ascending (vz, vy, vx, point index);
 * a point's neighbours are ranked by the FP32 squared distance
 * fmaf(dx, dx, fmaf(dy, dy, dz * dz)), ties to the lower index; the field's
 * key of a point for cell c is e^T e in FP32 ((ex ex + ey ey) + ez ez), e = p -
 * ((float)c + 0.5) r, ties to the smaller id.
 * Errors: MP_E_ARG for n < 0, null, non-finite or out-of-range coordinates
 * (|p / r| >= 2^30) or bad params; MP_E_UNSUPPORTED when the band grid exceeds
 * 2^32 - 2 cells (hash) or 2^27 - 2 cells or 2^24 cells per plane (dense), for
 * POINT with the HASH backend, and for POINT when the box of all map voxels
 * exceeds 2^28 cells.  n = 0 builds an empty map (every lookup misses). */
MP_API mp_status mp_map_build(const float* xyz, int64_t n, const mp_map_params* params, void* stream, mp_map* out);

MP_API mp_status mp_map_get_info(mp_map map, mp_map_info* out);

/* Copy the Gaussians out: mu G x 3, normal G x 3 (unit eigenvector n of the
 * GICP normalisation), voxel G x 3 (int32), count G (int32).  Any pointer may
 * be null. */
MP_API mp_status mp_map_get_gauss(mp_map map, float* mu, float* normal, int32_t* voxel, int32_t* count, void* stream);

/* Nearest-neighbour field lookup of n points (the exact path the likelihood
 * kernel takes): gid_out[i] = Gaussian id or -1. */
MP_API mp_status mp_map_lookup(mp_map map, const float* xyz, int64_t n, int32_t* gid_out, void* stream);

/* MP_E_STATE while a filter still uses the map. */
MP_API mp_status mp_map_destroy(mp_map map);

/* --------------------------------------------------------------- filter */

typedef struct {
    int32_t n_particles;  /* N^P, 1 .. 2^26 */
    int32_t k;            /* K, neighbour-list length including the particle itself, 1..32 (Sec. III-C) */
    int32_t lsh_bits;     /* N^B = 2^lsh_bits buckets, 0..30 (Eq. 9, Alg. 1) */
    int32_t svgd_iters;   /* SVGD iterations per filter step, >= 0 */
    int32_t post_iters;   /* rounds of the neighbour-graph propagation (Eq. 11), >= 0 */
    int32_t window_c;     /* bucket-mates examined per particle and iteration, >= 0 */
    int32_t scan_k;       /* neighbours for scan covariances, 3..32 */
    float sigma_r;        /* W^K rotation weight, 1/rad (Eq. 7) */
    float sigma_t;        /* W^K translation weight, 1/m */
    float lsh_alpha;      /* alpha of Eq. 10 */
    float lsh_sigma;      /* per-axis std of delta^LSH, in cells (Eq. 10) */
    float c_max;          /* per-point cost cap; outliers cost c_max */
    float d_max;          /* inlier gate on |mu^M - T mu^S|, metres */
    float lambda_rel;     /* Marquardt damping of the GN step: H + diag(lambda_rel H_ii + lambda_abs) */
    float lambda_abs;
    float temperature;    /* log-likelihood divisor in the posterior */
    float prior_floor;    /* prior probabilities below this are raised to it */
    float cov_eps;        /* GICP epsilon for scan covariances */
    int32_t lik_chunks;   /* scan-point chunks per particle tile in the likelihood launch; 0 = auto */
    int32_t lik_batch;    /* scan points whose NNF cells are requested together per lane: 1..32 (power of 2);
                             0 = 4 in the PARTICLE layout, 2 in the GROUPED one (GROUPED takes 2, 4 or 8) */
    int32_t lik_layout;   /* MP_LIK_LAYOUT_*: lanes per particle in the likelihood launch */
    int32_t scorer;       /* MP_SCORER_*: per-point term of the likelihood */
    float sigma_s;        /* MP_SCORER_SCOREFIELD: isotropic sensor std of the score field, metres */
    int32_t lsh_tangent;  /* MP_LSH_TANGENT_*: tangent of T_i at T^LSH that Eq. (10) hashes */
    int32_t lsh_tables;   /* hash tables per SVGD iteration, 0..16 (0 = 1): each draws its own T^LSH and
                             delta^LSH and refreshes the neighbour lists once */
    int32_t svgd_grad;    /* MP_SVGD_GRAD_*: kernel gradient in the update of Eq. (5)-(6) */
    int32_t svgd_transport; /* MP_SVGD_TRANSPORT_*: tangent frame of neighbour j's term */
    int32_t final_rescore;  /* 1: after the last SVGD update, evaluate the likelihood and the kernel
                               values of the lists again at the final poses, so that the posterior
                               (Sec. III-D) scores the poses it reports; 0: it scores the last
                               iteration's (pre-update) likelihoods, as the paper's step order does */
    uint64_t seed;        /* Philox4x32-10 key */
} mp_filter_params;

/* Tangent hashed by the LSH (Eq. 10), x_i with zeta = alpha W^K x_i + delta_i:
 *   DECOUPLED  [log(R_L^T R_i); R_L^T (t_i - t_L)]  (rotation vector and
 *              rotated translation offset);
 *   SE3        log(T_LSH^-1 T_i), the coupled SE(3) logarithm of Eq. (8)
 *              (same rotation part; translation V(omega)^-1 R_L^T (t_i - t_L)). */
enum { MP_LSH_TANGENT_DECOUPLED = 0, MP_LSH_TANGENT_SE3 = 1 };

/* Kernel gradient of the Stein update, with respect to a right perturbation
 * of T_j (Eq. 5-8):
 *   APPROX  -2 k_ij W^K d_ij   (the inverse right Jacobian of the logarithm
 *           taken as the identity);
 *   EXACT   -2 k_ij J_r^-1(d_ij)^T W^K d_ij, J_r^-1 in closed form. */
enum { MP_SVGD_GRAD_APPROX = 0, MP_SVGD_GRAD_EXACT = 1 };

/* Frame of neighbour j's term k_ij psi_j + grad in the sum for particle i:
 *   NONE     added as it is;
 *   ADJOINT  carried from the tangent at T_j to the tangent at T_i by
 *            Ad_{T_i^-1 T_j} = [[R, 0], [t^ R, R]] of T_i^-1 T_j = (R, t). */
enum { MP_SVGD_TRANSPORT_NONE = 0, MP_SVGD_TRANSPORT_ADJOINT = 1 };

/* Per-point term of the likelihood.
 *   PLAIN       the GICP cost of Eq. (3) with full Gauss-Newton H, b (Eq. 4).
 *   SCOREFIELD  the residual field of the transformed point p' (scan
 *               covariances unused): inside the gate (NNF hit, |e| <= d_max)
 *               s = e^T (Sigma^M + sigma_s^2 I)^-1 e untruncated, r = sqrt(s),
 *               grad r = grad s / (2 max(r, 1e-2)); outside r = r_out =
 *               d_max / sqrt(cov_eps + sigma_s^2) and grad r = 0.  Rank-1
 *               Gauss-Newton: g = J^T grad r (J = dp'/d delta), H += g g^T,
 *               b += r g; log-likelihood -min(r^2, c_max).
 *   SURROGATE   the same with r and grad r predicted by a trained network
 *               (mp_surrogate_*), attached by mp_filter_set_surrogate.
 * Points with r^2 >= c_max are counted as outliers. */
enum { MP_SCORER_PLAIN = 0, MP_SCORER_SCOREFIELD = 1, MP_SCORER_SURROGATE = 2 };

/* Likelihood launch layout (results agree to rounding; the choice is speed):
 *   PARTICLE  one lane per particle, 256 particles per workgroup, scan tiles
 *             broadcast from LDS (suits few particles or short scans);
 *   GROUPED   16 lanes per particle walking consecutive scan points, so a
 *             wave's gathers fall in a few compact clusters of map cells;
 *             scan chunks of 1024 points held in LDS (lik_chunks ignored);
 *   AUTO      GROUPED when N >= 2048 and the scan has >= 512 points. */
enum { MP_LIK_LAYOUT_AUTO = 0, MP_LIK_LAYOUT_PARTICLE = 1, MP_LIK_LAYOUT_GROUPED = 2 };

/* Defaults: k 16, lsh_bits 20, svgd_iters 10, post_iters 10, window_c 32,
 * scan_k 10, sigma_r 5, sigma_t 2.5, lsh_alpha 1, lsh_sigma 0.3, c_max 9,
 * d_max 1.0, lambda_rel 1e-3, lambda_abs 1e-6, temperature 1,
 * prior_floor 1e-30, cov_eps 1e-3, lik_chunks 0, lik_batch 0, lik_layout AUTO,
 * scorer PLAIN, sigma_s 0.03, lsh_tangent DECOUPLED, lsh_tables 1, svgd_grad
 * APPROX, svgd_transport NONE, final_rescore 0, seed 1. */
MP_API void mp_filter_default_params(mp_filter_params* p);

enum { MP_INIT_UNIFORM_BOX = 0, MP_INIT_EXPLICIT = 1, MP_INIT_GAUSSIAN = 2 };

typedef struct {
    int32_t kind;        /* MP_INIT_* */
    float box_min[3];    /* UNIFORM_BOX: translation box; rotation uniform on SO(3) */
    float box_max[3];
    const float* poses;  /* EXPLICIT: n_particles x 7 (host or device) */
    float mean[7];       /* GAUSSIAN: pose M the particles spread about */
    float cov[36];       /* GAUSSIAN: 6 x 6 covariance (row-major, tangent [omega; v]) */
} mp_init_desc;

/* Create a filter on `map`: N particles, prior 1/N, neighbour lists {i},
 * frame 0 (Sec. III-A).  Uniform poses come from Philox(seed) with Shoemake's
 * uniform rotations, so they are reproducible.  Explicit quaternions are
 * normalised on input.  Gaussian poses are M exp(L z_i) with L L^T = cov and
 * z_i ~ N(0, I6) from Philox(seed; i), drawn like the prediction noise of
 * Eq. (1) (a tracking start about a known pose).  Errors: MP_E_ARG (params
 * out of range, non-finite or zero quaternions, a covariance that is not
 * symmetric positive semi-definite), MP_E_OOM. */
MP_API mp_status mp_filter_init(mp_map map, const mp_filter_params* params, const mp_init_desc* init, void* stream,
                         mp_filter* out);

MP_API mp_status mp_filter_destroy(mp_filter f);

/* Upload the scan P_t (Sec. III-A) for the next filter steps.
 *   xyz  n x 3 float32 points in the sensor frame.
 *   cov6 n x 6 (xx, xy, xz, yy, yz, zz) scan covariances or NULL: then each
 *        point gets the GICP-normalised covariance of itself and its scan_k
 *        nearest scan points (ties to the lower index) (Sec. III-C, Segal et
 *        al. 2009).
 * n = 0 is legal (occlusion): steps then only predict.  Errors: MP_E_ARG for
 * n < 0, null with n > 0, n > 65536 or non-finite values. */
MP_API mp_status mp_scan_upload(mp_filter f, const float* xyz, const float* cov6, int32_t n, void* stream);

/* One filter step.
 *   Prediction (Eq. 1): T_i <- T_i dT exp(delta_i), delta_i ~ N(0, cov_dT)
 *   drawn from Philox(seed; i, frame).  dT = NULL skips prediction; cov_dT =
 *   NULL means no noise.  cov_dT is 6x6 row-major over [omega; v], symmetric
 *   positive semi-definite.
 *   Correction, svgd_iters times: LSH bucketing and neighbour-list refresh
 *   (Eq. 9-10, Alg. 1), likelihood with Gauss-Newton H, b and psi (Eq. 2-4),
 *   SVGD update over the neighbour lists (Eq. 5-8).
 *   Posterior (Eq. 11): prior x likelihood of the last iteration, FP64
 *   log-sum-exp, post_iters propagation rounds, renormalisation, argmax.
 * Asynchronous; nothing synchronises the host.  Errors: MP_E_STATE before the
 * first mp_scan_upload, MP_E_ARG for non-finite dT/cov_dT or a covariance that
 * is not positive semi-definite, MP_E_OOM when the step's work buffers (sized
 * by the particle count and the scan: 116 bytes per particle per 1024 scan
 * points for the likelihood's partial sums) cannot be allocated; in every
 * error case nothing has been launched and the filter is unchanged. */
MP_API mp_status mp_filter_step(mp_filter f, const float dT[7], const float cov_dT[36], void* stream);

typedef struct {
    float map_pose[7];     /* pose of the maximum-posterior particle (Sec. III-D) */
    int32_t map_index;     /* its index */
    double map_weight;     /* its posterior probability */
    double n_eff;          /* 1 / sum p^2 */
    double log_evidence;   /* log sum_i exp(l_i) before normalisation */
    double max_loglik;     /* largest log-likelihood of the last iteration */
    int32_t frame;         /* filter steps taken */
    int32_t fp64_resolves; /* Gauss-Newton solves redone in FP64 in the last step */
    int32_t fallback_steps; /* steps the SURROGATE scorer ran as PLAIN (mp_filter_set_surrogate_check) */
    int32_t sur_checks;    /* surrogate checks made */
    float sur_check_ds;    /* mean |delta s| of the last check, -1 before the first */
} mp_posterior;

/* Read the representative state and, optionally, all poses (N x 7) and the
 * posterior weights (N, FP64).  Synchronises `stream`.  MP_E_NUMERIC if a
 * pose or weight is not finite; unlike other errors, the requested outputs
 * are still written then, so that the caller can find the particle. */
MP_API mp_status mp_posterior_query(mp_filter f, mp_posterior* out, float* poses_out, double* weights_out, void* stream);

/* Message of the last failing call on this thread ("" if none). */
MP_API const char* mp_last_error(void);

/* ----------------------------------------------------------- diagnostics */

enum {
    MP_STAGE_PREDICT = 0,  /* Eq. 1 */
    MP_STAGE_LSH = 1,      /* Eq. 9-10: codes */
    MP_STAGE_SORT = 2,     /* Alg. 1 distribute loop: stable sort + bucket bounds */
    MP_STAGE_REFRESH = 3,  /* Alg. 1 gather loop: neighbour refresh + kernel values */
    MP_STAGE_LIK = 4,      /* Eq. 2-4: likelihood, H, b, psi */
    MP_STAGE_SVGD = 5,     /* Eq. 5-8 */
    MP_STAGE_POSTERIOR = 6,/* Eq. 11 */
    MP_STAGE_SCAN = 7,     /* scan covariances (mp_scan_upload) */
    MP_STAGE_LIK_CORE = 8, /* the likelihood accumulation kernel alone (inside MP_STAGE_LIK) */
    MP_NUM_STAGES = 9
};

/* Per-stage device time of the last mp_filter_step (scan stage: of the last
 * mp_scan_upload), milliseconds, summed over the step's iterations, from HIP
 * event pairs recorded on the call's stream around each stage's launches
 * (synchronises).  ms_out has MP_NUM_STAGES entries; stages not run read 0.
 * counts_out (nullable, MP_NUM_STAGES) receives the number of timed spans. */
MP_API mp_status mp_stage_times(mp_filter f, float* ms_out, int32_t* counts_out);

/* Test-only access to the filter state, by name, in the library's own layout:
 *   "poses"   N x 8 float (qw,qx,qy,qz,tx,ty,tz,0), current buffer
 *   "psi"     N x 8 float (psi[6], loglik, inlier count as float)
 *   "hb"      N x 28 float (H upper 21 row-major, b 6, cost) of the last
 *             likelihood pass; only written after set "capture_hb" = 1
 *   "solve"   N int32, how the last pass solved each psi (written with "hb"):
 *             0 FP32 Cholesky, 1 FP64 re-solve (FP32 failed or its condition
 *             estimate exceeded 1e6), 2 both failed (psi = 0)
 *   "codes"   N uint32 LSH codes of the last LSH pass (particle order)
 *   "sorted"  N int32 particle index at each sorted position
 *   "scodes"  N uint32 codes in sorted order
 *   "head", "end"  N int32 bucket bounds per sorted position
 *   "nbr"     K x N int32 neighbour lists (column-major, -1 pads)
 *   "kval"    K x N float kernel values k_ij (0 for pads)
 *   "cnt"     N int32 list lengths
 *   "prior"   N float prior probabilities
 *   "post"    N float smoothed posterior of the last step
 *   "scan"    n x 12 float scan records (mu, Sigma upper 6, pad), caller's order
 *   "scan_walk" the same records in the likelihood's walk order (Morton order
 *             of the points on a grid of half the map voxel)
 *   "tlsh"    8 float T^LSH of the last LSH pass
 *   "sort_wait" uint32, 0 after a good bucket sort; 1 if a workgroup of the
 *             last one stopped waiting for the digit counts of the tiles
 *             before it (its wait is bounded), 2 if a key's sorted place fell
 *             outside the output (keys changed during the sort); then that
 *             sort's order is wrong
 *   "capture_hb"  int32 (set only)
 * bytes must equal the named buffer's size.  mp_debug_stage runs one stage
 * on the current state (iteration selects the LSH frame counter; dT/cov_dT as
 * in mp_filter_step, used by MP_STAGE_PREDICT only); MP_DEBUG_RESCORE runs
 * the final re-score of a step with final_rescore (a likelihood pass and a
 * refresh that only re-ranks the current lists). */
enum { MP_DEBUG_RESCORE = 100 };
MP_API mp_status mp_debug_get(mp_filter f, const char* name, void* dst, int64_t bytes, void* stream);
MP_API mp_status mp_debug_set(mp_filter f, const char* name, const void* src, int64_t bytes, void* stream);
MP_API mp_status mp_debug_stage(mp_filter f, int32_t stage, int32_t iteration, const float dT[7], const float cov_dT[36],
                         void* stream);

/* Test output of the per-point map construction (Sec. III-C, per-point
 * Gaussians): builds a POINT map from xyz as mp_map_build does, writes each
 * point's neighbour list, knn_out[i * point_k + a] = index of its a-th nearest
 * other point in the order the build ranks them (FP32 squared distance, ties
 * to the lower index), -1 pads, and frees the map.  xyz n x 3 float32 and
 * knn_out n x point_k int32 are host or device pointers; synchronises.
 * Errors: MP_E_ARG for a null pointer, n <= 0 or a gauss_mode other than
 * POINT, and every error of mp_map_build. */
MP_API mp_status mp_debug_map_point_knn(const float* xyz, int64_t n, const mp_map_params* params, int32_t* knn_out,
                                        void* stream);

/* Test access to the stable radix sort that distributes particles into LSH
 * buckets (Alg. 1, distribute loop): sorts keys[0..n), each below 2^bits
 * (bits 1..32; the sort makes one pass per 8 bits), equal keys keeping their
 * input order, and writes the sorted keys to keys_out and, for each sorted
 * position, the input index of its key to order_out.  keys (n uint32), keys_out (n uint32) and
 * order_out (n int32) are host or device pointers; synchronises.  Errors:
 * MP_E_ARG for a null pointer, n <= 0 or bits outside 1..32,
 * MP_E_UNSUPPORTED for n >= 2^30, MP_E_HIP if a workgroup stopped waiting
 * for the digit counts of the tiles before it (its wait is bounded) or a
 * key's place fell outside the output. */
MP_API mp_status mp_debug_sort_u32(const uint32_t* keys, int64_t n, int32_t bits, uint32_t* keys_out,
                                   int32_t* order_out, void* stream);

/* ------------------------------------------------------------ batch */
/* Several independent filters (instances: different maps, particle counts,
 * scans and parameters) stepped by one call.  The first step captures every
 * instance's whole filter step (prediction, correction iterations, posterior;
 * exactly the launches of mp_filter_step) into one HIP graph, each instance on
 * its own branch, and every call replays it: per-step values (frame counter,
 * odometry increment, noise factor) are uploaded to device memory before the
 * replay, so the graph itself never changes.  A new capture happens when an
 * instance's scan size or buffers changed (mp_scan_upload with another n).
 * Results equal those of mp_filter_step on each instance, bit for bit.
 * The filters stay usable alone; they cannot be destroyed while in a batch. */
typedef struct mp_batch_s* mp_batch;

typedef struct {
    int32_t n_instances;
    int32_t captures;        /* graphs captured so far */
    int64_t evals_per_step;  /* particle-point evaluations of one batch step */
    int32_t queued_instances;   /* instances whose likelihood runs in the tile queue (first iteration) */
    int32_t queue_batch;        /* gather batch of the queue kernel */
    int32_t queue_workgroups;   /* workgroups of the persistent launch */
    int32_t pad;
    int64_t queue_tiles_per_step; /* tiles (256 particles x 1024 scan points) per step through the queues */
} mp_batch_info;

/* Instances with the PLAIN scorer on a dense-field map get lik_layout =
 * GROUPED: in every correction iteration their likelihood passes run as one
 * persistent launch (a fixed grid of workgroups taking tiles of 256 particles
 * x 1024 scan points of all these instances, in instance order, from an
 * atomic work queue); the other instances launch their own
 * likelihood kernels on their branch.  autotune != 0 times the queue kernel
 * for each gather batch (2, 4, 8) and keeps the fastest, and times the
 * likelihood launch of every other PLAIN instance for each (lik_layout,
 * lik_batch) candidate (PARTICLE with 2, 4, 8, 16; GROUPED with 2, 4, 8) and
 * keeps the fastest in its parameters (speed only: the per-point arithmetic is
 * the same; sums are ordered differently by the two layouts).  Every filter
 * needs a scan uploaded.  Errors: MP_E_ARG, MP_E_STATE (no scan, a filter
 * given twice, SURROGATE scorer without a network). */
MP_API mp_status mp_batch_create(const mp_filter* filters, int32_t n, int32_t autotune, void* stream, mp_batch* out);

/* One step of every instance.  dT: n x 7 (NULL: no prediction for any
 * instance); cov_dT: n x 36 (NULL: no noise); as in mp_filter_step.  Host
 * arrays.  Asynchronous except for waiting until the previous call's step
 * values have been copied. */
MP_API mp_status mp_batch_step(mp_batch b, const float* dT, const float* cov_dT, void* stream);

/* lik_batch_out, lik_layout_out (nullable): the n instances' values in use. */
MP_API mp_status mp_batch_get_info(mp_batch b, mp_batch_info* out, int32_t* lik_batch_out, int32_t* lik_layout_out);

MP_API mp_status mp_batch_destroy(mp_batch b);

/* ------------------------------------------------------------ surrogate */
/* A learned replacement of the map's per-point residual (the residual field of
 * MP_SCORER_SCOREFIELD) by a small network evaluated on the matrix cores:
 *   x = (p - box_min) / L, L = the box's largest extent;
 *   features sin, cos(2 pi frac(f_l x_a)), f_l = f_max^(l/31), l = 0..31,
 *   per axis a, ordered (axis, frequency, sin|cos): 192 inputs;
 *   192 -> 128 -> 128 -> 4, SiLU after the two hidden layers;
 *   outputs (r / r_scale, grad r / g_scale) of the residual field of
 *   MP_SCORER_SCOREFIELD, r_scale = r_out = d_max / sqrt(eps + sigma_s^2) and
 *   g_scale = 1 / sqrt(eps + sigma_s^2) (the largest |grad r|), eps the
 *   map's cov_eps.
 * Products take bfloat16 operands with FP32 accumulation; weights are kept
 * in FP32 (master) with bfloat16 copies; training is Adam on the mean squared
 * error of the 4 scaled outputs against residual-field labels. */
typedef struct mp_surrogate_s* mp_surrogate;

#define MP_SUR_NPARAMS 41732       /* 192*128 + 128 + 128*128 + 128 + 128*4 + 4 */
#define MP_SUR_IMAGE_BYTES 84112   /* inference weights as held in LDS */

typedef struct {
    float box_min[3], box_max[3];  /* feature box; box_min == box_max: the map's voxel box */
    float f_max;          /* highest frequency, cycles per L; 0: L / voxel */
    float sigma_s;        /* score-field sensor std, metres */
    float d_max, c_max;   /* inlier gate (0: two voxels); c_max is kept for reference (the scorer uses the filter's) */
    float lr, lr_min;     /* Adam step, cosine-decayed from lr to lr_min over total_steps */
    float beta1, beta2, adam_eps;
    int32_t total_steps;  /* length of the cosine schedule */
    int32_t batch;        /* samples per Adam step, 256 .. 2^20 */
    uint64_t seed;        /* Philox key of the initial weights and the batch draws */
} mp_surrogate_params;

typedef struct {
    int64_t n_params;       /* 41732 */
    int64_t n_data;         /* training samples held */
    int64_t steps;          /* Adam steps taken */
    float lo[3], inv_ext[3];/* feature normalisation x = (p - lo) * inv_ext (FP32) */
    float freqs[32];        /* f_l, cycles per normalised unit (FP32) */
    float r_scale, g_scale; /* output scales */
    int32_t weight_bytes;   /* bytes of the inference image held in LDS per workgroup */
} mp_surrogate_info;

/* Defaults: box from the map, f_max 0, sigma_s 0.03, d_max 0, c_max 9,
 * lr 1e-3, lr_min 1e-5, betas 0.9 / 0.999, eps 1e-8, total_steps 20000,
 * batch 65536, seed 1. */
MP_API void mp_surrogate_default_params(mp_surrogate_params* p);

/* Create a network for `map` (which must outlive it).  Weights are drawn
 * uniform in +-1/sqrt(fan_in) from Philox(seed), biases zero.  Errors:
 * MP_E_ARG (bad params), MP_E_OOM. */
MP_API mp_status mp_surrogate_create(mp_map map, const mp_surrogate_params* params, void* stream, mp_surrogate* out);

/* MP_E_STATE while a filter still uses the network. */
MP_API mp_status mp_surrogate_destroy(mp_surrogate sur);

MP_API mp_status mp_surrogate_get_info(mp_surrogate sur, mp_surrogate_info* out);

/* Exact residual-field labels of n points: out4 = (r, grad r) per point,
 * n x 4 float, physical units (the training targets before scaling). */
MP_API mp_status mp_surrogate_label(mp_surrogate sur, const float* xyz, int64_t n, float* out4, void* stream);

/* Network prediction of n points: out4 = (r, grad r), n x 4 float, physical
 * units, unclamped. */
MP_API mp_status mp_surrogate_eval(mp_surrogate sur, const float* xyz, int64_t n, float* out4, void* stream);

/* Replace the training set by n points (n x 3); labels are computed on the
 * device.  n >= 1. */
MP_API mp_status mp_surrogate_set_data(mp_surrogate sur, const float* xyz, int64_t n, void* stream);

/* Take `steps` Adam steps.  Each batch is `batch` samples drawn uniformly
 * with replacement from the training set by Philox(seed; step); when the set
 * holds no more than `batch` samples every step uses the whole set.
 * loss_out (host, nullable) receives each step's loss and makes the call
 * synchronous.  Errors: MP_E_STATE without training data. */
MP_API mp_status mp_surrogate_train(mp_surrogate sur, int32_t steps, float* loss_out, void* stream);

/* Loss and gradient of the current weights over n given samples with given
 * targets (n x 4, physical units), without an update.  grad_out: n_params
 * float (host or device) in the parameter layout below; loss_out: host float.
 * n <= batch. */
MP_API mp_status mp_surrogate_grad(mp_surrogate sur, const float* xyz, const float* target4, int64_t n,
                                   float* grad_out, float* loss_out, void* stream);

/* FP32 weights in the layout W1[192][128], b1[128], W2[128][128], b2[128],
 * W3[128][4], b3[4] (input-major matrices).  Setting them clears the Adam
 * moments and the step count. */
MP_API mp_status mp_surrogate_get_params(mp_surrogate sur, float* params, void* stream);
MP_API mp_status mp_surrogate_set_params(mp_surrogate sur, const float* params, void* stream);

/* Attach (or detach with NULL) the network the filter's SURROGATE scorer
 * uses; the network must outlive the attachment. */
MP_API mp_status mp_filter_set_surrogate(mp_filter f, mp_surrogate sur);

/* ------------------------------------------------------------ odometry */

/* GICP scan-to-scan odometry (Sec. III-B): the sensor motion dT between the
 * filter's previous and current scan (the last two non-empty mp_scan_upload
 * calls) and its covariance from the Hessian of the match, the dT and
 * Sigma^dT that mp_filter_step's prediction takes (Eq. 1).  dT maps points of
 * the current scan's frame into the previous scan's frame (T_t = T_{t-1} dT).
 * Each scan point p_k = R mu_k + t is matched to the nearest point of the
 * previous scan (FP32 squared distance, ties to the lower index; a match
 * farther than d_max is dropped); GICP term with C = T_j + R S_k R^T (both
 * scans' GICP-normalised covariances); `iterations` damped Gauss-Newton
 * updates dT <- dT exp(psi) with the filter's damping; then
 * Sigma^dT = cov_scale * H^-1 at the final pose (the paper gives no scale;
 * with GICP-normalised covariances H^-1 is in units of the normalised
 * residuals, so the scale sets the prediction noise). */
typedef struct {
    int32_t iterations;   /* Gauss-Newton updates, 0..1000 (0: evaluate at the initial dT) */
    float d_max;          /* correspondence gate, metres, > 0 */
    float lambda_rel;     /* damping: H_ii (1 + lambda_rel) + lambda_abs */
    float lambda_abs;
    float cov_scale;      /* Sigma^dT = cov_scale * H^-1, > 0 */
} mp_odometry_params;

typedef struct {
    double H[21];         /* GICP Hessian at the final dT (upper triangle, row-major, [omega; v]) */
    double b[6];          /* gradient there */
    double cost;          /* sum of e^T Omega e over the matches */
    int32_t inliers;      /* matches within d_max */
    int32_t iterations;
    int32_t cov_ok;       /* 0 if H was not positive definite (covariance zeroed) */
    double dT64[7];       /* the final dT before rounding to FP32 */
} mp_odometry_result;

/* Defaults: iterations 20, d_max 1.0, lambda_rel 1e-3, lambda_abs 1e-6,
 * cov_scale 1. */
MP_API void mp_odometry_default_params(mp_odometry_params* p);

/* init_dT (nullable: identity) is the starting motion; dT_out (7 floats,
 * required), cov_out (36 floats, nullable, row-major over [omega; v]) and
 * result (nullable) are host pointers; synchronises the stream.  Errors:
 * MP_E_ARG (null filter / params / dT_out, parameters out of range, non-finite
 * or zero-quaternion init_dT), MP_E_STATE (fewer than two non-empty scans
 * uploaded). */
MP_API mp_status mp_odometry(mp_filter f, const mp_odometry_params* params, const float init_dT[7], float dT_out[7],
                             float cov_out[36], mp_odometry_result* result, void* stream);

/* mp_odometry for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and results, bit for bit, with its work arrays (match
 * keys, matches, per-workgroup sums, the pose state) in a fixed device area
 * of 0.21 MB that the library holds on each device it runs on until the
 * process ends; no hipMalloc, hipFree or allocating library call.  The filter's scans are the
 * inputs, the host outputs as in mp_odometry.  The current scan may hold at
 * most 16384 points (MP_E_ARG beyond).  Every call on a device shares that
 * device's area: calls that overlap on one device (several host threads or
 * streams) race and must be serialised by the caller.  Errors: those of
 * mp_odometry. */
MP_API mp_status mp_odometry_noalloc(mp_filter f, const mp_odometry_params* params, const float init_dT[7],
                                     float dT_out[7], float cov_out[36], mp_odometry_result* result, void* stream);

/* ------------------------------------------------------------ smoothing */

/* Smoothing of the representative pose (Sec. IV-A: the maximum-posterior
 * particle jitters from frame to frame; simple trajectory smoothing removes
 * it).  Host code, no GPU work.  mp_smoother_push takes a frame's
 * representative pose (e.g. mp_posterior.map_pose) and the motion dT since
 * the previous push (nullable: none).  The track keeps the last `window`
 * accepted poses, each carried forward by the reported motion (T <- T dT).
 * A pose within jump_m / jump_rad of the carried newest one is accepted; a
 * farther one (the maximum on another mode for a frame, or a recovery after
 * a kidnap) is held back until switch_frames consecutive far poses agree
 * with each other, which then replace the track.  The output is
 * T_new exp(mean_i log(T_new^-1 T_i)) over the track (FP64 inside). */
typedef struct {
    int32_t window;        /* poses averaged, 1..1024 */
    float jump_m;          /* a pose farther than this translation, metres (> 0), */
    float jump_rad;        /* ... or this rotation, radians (> 0), is far */
    int32_t switch_frames; /* consecutive agreeing far poses that move the track, 1..1024 */
} mp_smoother_params;
typedef struct mp_smoother_s* mp_smoother;

/* Defaults: window 5, jump_m 1.0, jump_rad 0.2, switch_frames 3. */
MP_API void mp_smoother_default_params(mp_smoother_params* p);
/* Errors: MP_E_ARG (null, window, switch_frames or thresholds out of range), MP_E_OOM. */
MP_API mp_status mp_smoother_create(const mp_smoother_params* params, mp_smoother* out);
/* pose, dT, out: host arrays of 7 floats (qw qx qy qz tx ty tz).  Errors:
 * MP_E_ARG (null smoother / pose / out, non-finite values, zero quaternion). */
MP_API mp_status mp_smoother_push(mp_smoother s, const float pose[7], const float dT[7], float out[7]);
MP_API mp_status mp_smoother_destroy(mp_smoother s);

/* Check of the SURROGATE scorer against the exact residual field it
 * approximates (a safeguard of the learned configuration, not of the paper):
 * when a filter step starts at a multiple of `period` steps (period 0, the
 * default, turns the check off) and no fallback is running, the scan points
 * transformed by every `stride`-th particle (walk order, thinned to at most
 * 2^22 pairs) are scored by the network and by the exact field; if the mean
 * |min(r_net^2, c_max) - min(r^2, c_max)| exceeds `threshold` (or is not a
 * number), that step and the next fallback - 1 run the PLAIN scorer.  Each
 * check synchronises the stream once; mp_posterior reports the steps run as
 * PLAIN, the checks made and the last mean difference.  Example: period 10,
 * stride 100 (1% of the particles), threshold 0.5, fallback 10.  A filter with
 * the check on cannot join a batch (mp_batch_create: MP_E_UNSUPPORTED).
 * Errors: MP_E_ARG (period < 0, stride < 1, fallback < 0, threshold negative
 * or not finite), MP_E_STATE (filter held by a batch). */
MP_API mp_status mp_filter_set_surrogate_check(mp_filter f, int32_t period, int32_t stride, float threshold,
                                               int32_t fallback);

#ifdef __cplusplus
}
#endif

#endif /* MEGAPF_H */
