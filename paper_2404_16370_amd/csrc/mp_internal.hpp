// mp_internal.hpp -- library-internal structures and stage launchers.
#pragma once
#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "megapf.h"

// ------------------------------------------------------------ errors
struct MpError {
    mp_status code;
    std::string msg;
};

[[noreturn]] void mp_throw(mp_status code, const char* fmt, ...);

#define MP_HIP(expr)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess) {                                                                       \
            if (_e == hipErrorOutOfMemory) mp_throw(MP_E_OOM, "%s: %s", #expr, hipGetErrorString(_e)); \
            mp_throw(MP_E_HIP, "%s: %s", #expr, hipGetErrorString(_e));                               \
        }                                                                                             \
    } while (0)

#define MP_CHECK_LAUNCH() MP_HIP(hipGetLastError())

// ------------------------------------------------------------ device memory
// Owning device allocation; freed in the destructor.
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void alloc(size_t b);          // exact size, contents undefined
    void ensure(size_t b);         // grow if smaller
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
    void swap(DevMem& o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
};

// ------------------------------------------------------------ map
// What the likelihood kernel needs to look up the nearest-neighbour field
// and read the Gaussians; passed to kernels by value.
struct MapView {
    float inv_r;         // 1/r in FP32
    float gicp_a;        // 1 - eps: Sigma^M = I - a n n^T
    int32_t org[3];      // band grid origin (voxel coordinates)
    int32_t dim[3];      // band grid extent
    int32_t backend;     // MP_NNF_HASH or MP_NNF_DENSE
    uint32_t mask;       // hash capacity - 1
    const int32_t* dense;   // dim product cells, -1 = miss
    const uint2* table;     // hash slots {key = linear index + 1 (0 empty), gid}
    const float4* gauss;    // 2 per Gaussian: (mu, count), (n, 0)
    const float4* drec;     // dense backend: 2 per cell, the nearest Gaussian's record
                            // (cells outside the band: a far sentinel mean), then one
                            // more record (index dmiss) for points outside the grid
    uint32_t dxy;           // dense backend: dim[0] * dim[1] (< 2^24)
    uint32_t dmiss;         // dense backend: cells of the grid (< 2^27 - 1)
};

struct mp_map_s {
    mp_map_params params{};
    mp_map_info info{};
    MapView view{};
    DevMem gauss, dense, drec, table, vox;   // vox: G x int3 voxel coordinates
    float box_lo[3], box_hi[3];
    int users = 0;
    int32_t* knn_dbg = nullptr;   // test output of the per-point build: n x point_k lists (device), or null
};

// ------------------------------------------------------------ surrogate
struct mp_surrogate_s {
    mp_map map = nullptr;
    mp_surrogate_params p{};
    mp_surrogate_info info{};
    DevMem P, Mo, Vo, G;            // FP32 weights, Adam moments, last gradient
    DevMem img;                     // inference image (bf16 fragments, FP32 biases and frequencies)
    DevMem img2;                    // W2 fragments of the training's input-gradient product
    DevMem w3b;                     // bf16 copy of W3 (training's output-layer gradient)
    DevMem dxyz, dlab;              // training set: points, scaled labels (float4)
    int32_t cap = 0;                // padded batch rows the work buffers hold
    DevMem bxyz, btgt;              // a batch staged by the caller (mp_surrogate_grad)
    DevMem pf;                      // per-workgroup partial gradients of the training step
    DevMem losses;                  // per-step loss (float)
    int cus = 1;                    // compute units of the device (persistent-grid size)
    int users = 0;
};

// ------------------------------------------------------------ filter
// Values that change from one filter step to the next.  Kernels captured in a
// graph read them from device memory, written before each replay; eager
// launches pass them as kernel arguments instead.
struct StepDyn {
    uint32_t frame;      // filter step index: prediction and LSH counters
    int32_t do_pred;     // 0: this step has no prediction
    int32_t noise;       // prediction noise on
    int32_t pad;
    float dq[4], dt[4];  // odometry increment (quaternion w, x, y, z; translation)
    float L[24];         // packed lower-triangular noise factor (21 used)
};

struct FilterParamsDev {
    int32_t n, k, bits, window_c;
    float sigma_r, sigma_t, lsh_alpha, lsh_sigma, c_max, d_max, lambda_rel, lambda_abs;
    uint64_t seed;
};

// Check of the SURROGATE scorer against the exact residual field (off while
// period is 0): every `period` steps; fall back to PLAIN for `fallback` steps
// when the mean score difference exceeds `threshold`.
struct SurCheck {
    int32_t period = 0, stride = 100, fallback = 10;
    float threshold = 0.5f;
    int32_t left = 0;              // steps still to run with the PLAIN scorer
    int32_t fallback_steps = 0;    // steps run with PLAIN in place of SURROGATE
    int32_t checks = 0;
    float last = -1.0f;            // mean |delta s| of the last check
};

struct mp_filter_s {
    mp_map map = nullptr;
    mp_surrogate sur = nullptr;   // network of the SURROGATE scorer
    SurCheck chk;
    bool sur_fallback = false;    // this step: SURROGATE scorer replaced by PLAIN
    DevMem chk_buf;               // work arrays of the check
    const StepDyn* dyn = nullptr; // set while a step is captured into a graph
    bool capturing = false;       // no timers, no host work that a graph cannot hold
    int batch_users = 0;          // batches holding this filter
    mp_filter_params p{};
    hipStream_t last_stream = nullptr;
    int32_t n = 0, K = 0;
    int32_t frame = 0;
    int32_t lsh_counter = 0;  // frame value used by the LSH counter of the next pass
    int32_t scan_n = -1;      // -1: no scan uploaded yet
    int32_t cur = 0;          // current pose buffer
    int32_t capture_hb = 0;
    int32_t lik_chunks = 1, lik_chunk_len = 0;
    float lsh_lo[3], lsh_hi[3];
    // state
    DevMem poses[2];          // N x 8 float
    DevMem psi;               // N x 8 float: psi[6], loglik, inliers
    DevMem hb;                // N x 28 float (debug)
    DevMem solve_how;         // N int32 (debug): 0 FP32 Cholesky, 1 FP64 re-solve, 2 both failed (psi = 0)
    DevMem partial;           // chunks x 28 x N float
    DevMem codes, sorted, scodes, tmp_keys, tmp_vals, head, end, hist;  // LSH / sort
    DevMem lkeys, lorder;     // the likelihood's walk order: Morton keys, particle per position
    DevMem rank;   // sorted position of each particle (the refresh runs in particle order)
    DevMem nbr, kval, cnt;    // K x N, K x N, N
    DevMem prior, post0, post1;   // N float
    DevMem red;               // reduction scratch
    DevMem flags;             // per-step counters (int32)
    DevMem scan;              // n x 12 float records in the likelihood's walk order
    DevMem scan_orig;         // n x 12 float records in the caller's order
    DevMem scan_perm;         // n int32: walk position -> caller index
    DevMem scan_xyz;          // n x 3 float staging
    DevMem prev_orig;         // the previous non-empty scan's records (caller order), for odometry
    int32_t prev_n = 0;       // its points (0: none yet)
    int32_t orig_n = 0;       // points of the records in scan_orig (the last non-empty scan)
    DevMem odo_key, odo_nn, odo_part, odo_state;   // odometry work arrays
    DevMem scan_cov;          // n x 6 float staging of caller covariances
    DevMem scan_work;         // walk-order keys and work arrays (4n words) + lo/bad (4 floats)
    DevMem scan_sort;         // radix-sort scratch of the walk order
    DevMem tlsh;              // 8 float
    DevMem stepinfo;          // posterior summary (doubles)
    // stage timers: event pairs per stage and span, reused across steps
    std::vector<hipEvent_t> ev0[MP_NUM_STAGES], ev1[MP_NUM_STAGES];
    int ev_count[MP_NUM_STAGES] = {};
};

// record the start (begin = true) or end of span `ev_count[st]` of stage st
void mp_tick(mp_filter f, int st, bool begin, hipStream_t s);

// ------------------------------------------------------------ launchers
// sort / scan primitives (sort.hip)
void mp_scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, DevMem& scratch,
                           hipStream_t s);
// stable LSD radix sort of (key, value) by the low `bits` bits of the key;
// result in keys/vals (ping-pong with the alternate buffers)
void mp_radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s);
void mp_radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                       DevMem& scratch, hipStream_t s);
size_t mp_radix_scratch_bytes(int64_t n);
// number of 8-bit passes mp_radix_sort_* makes for n keys of `bits` bits
int mp_radix_passes(int64_t n, int bits);
// as mp_radix_sort_u32 without the final copy: after an odd number of passes
// the result is in (keys_alt, vals_alt)
void mp_radix_sort_u32_inplace_parity(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
                                      int bits, DevMem& scratch, hipStream_t s);
// device word of a 32-bit sort's scratch, zero after a good sort: 1 if a
// workgroup stopped waiting for its predecessors' counts, 2 if a key's place
// fell outside the output (its input changed while it ran); neither is
// expected, and the output of that sort is then wrong
uint32_t* mp_radix_wait_flag(DevMem& scratch);

// map (map_build.hip)
void mp_build_map(mp_map m, const float* xyz_dev, int64_t n, hipStream_t s);
void mp_map_lookup_launch(const MapView& v, const float* xyz_dev, int64_t n, int32_t* gid_dev, hipStream_t s);

// scan covariances (scan.hip)
void mp_scan_records(const float* xyz_dev, const float* cov6_dev, int32_t n, int32_t k, float eps, float* rec_dev,
                     hipStream_t s);
void mp_scan_permute(const float* rec_orig, const int32_t* perm, int32_t n, float* rec_out, hipStream_t s);
// lo_bad_dev (4 floats): bounding-box minimum corner of the points, then 1 if any
// point or covariance entry is not finite (else 0)
void mp_scan_check(const float* xyz_dev, const float* cov6_dev, int32_t n, float* lo_bad_dev, hipStream_t s);
// walk order of the likelihood: stable sort of the points by the Morton key of
// their cell (edge `cell`); keys/keys_alt/perm_alt are n-entry work arrays
void mp_scan_walk_order(const float* xyz_dev, int32_t n, float cell, const float* lo_bad_dev, uint32_t* keys,
                        uint32_t* keys_alt, int32_t* perm, int32_t* perm_alt, DevMem& scratch, hipStream_t s);

// filter stages
void mp_launch_init_uniform(mp_filter f, const float lo[3], const float hi[3], hipStream_t s);
// prediction T dT exp(L z); `gauss_init` draws z under the Gaussian-initialisation
// purpose instead of the prediction's (frame 0, at filter creation)
void mp_launch_predict(mp_filter f, const float dT[7], const float L[36], bool noise, hipStream_t s,
                       bool gauss_init = false);
void mp_launch_lsh(mp_filter f, uint32_t frame, uint32_t it, hipStream_t s);
void mp_launch_sort(mp_filter f, hipStream_t s);
// window < 0: the filter's window_c; 0 re-ranks the current lists at the current poses
void mp_launch_refresh(mp_filter f, hipStream_t s, int window = -1);
void mp_launch_likelihood(mp_filter f, hipStream_t s);
// Likelihood passes of several filters through one persistent tile queue
// (GROUPED layout, PLAIN scorer, dense field): the plan of a pass (false if it cannot
// join a queue; otherwise the pass's walk order is launched on s), the solve that
// follows the queue, the queue launch.
size_t mp_lik_args_bytes();
bool mp_lik_queue_plan(mp_filter f, void* args_out, int32_t* tiles, hipStream_t s);
void mp_lik_queue_solve(mp_filter f, hipStream_t s);
int mp_lik_queue_grid(int batch);
void mp_launch_lik_queue(const void* tab_dev, const int32_t* first_dev, int32_t* counter_dev, int n_inst, int tiles,
                         int batch, int grid, hipStream_t s);
// the phases of mp_step_launches (a batch interleaves them across filters)
void mp_step_begin(mp_filter f, bool pred, const float dq[7], const float L[36], bool noise, hipStream_t s);
void mp_step_iter_nbr(mp_filter f, int it, hipStream_t s);
void mp_step_iter_svgd(mp_filter f, int it, hipStream_t s);
void mp_step_end(mp_filter f, hipStream_t s);
void mp_launch_svgd(mp_filter f, hipStream_t s);
void mp_launch_posterior(mp_filter f, hipStream_t s);
void mp_launch_reset_lists(mp_filter f, hipStream_t s);
// device fill (graph-safe replacement of hipMemsetAsync)
void mp_fill_u32(void* p, uint32_t v, size_t n, hipStream_t s);
void mp_copy_poses(mp_filter f, int from, int to, hipStream_t s);
// size every buffer a step needs, so that a captured step allocates nothing
void mp_reserve_step(mp_filter f);
size_t mp_lik_partial_bytes(mp_filter f);
size_t mp_post_scratch_bytes(mp_filter f);
// the whole step on stream s (eager: dT/L as arguments; captured: from f->dyn)
// validate an odometry increment and factor its covariance (host)
void mp_prepare_prediction(const float dT[7], const float cov[36], float dq[7], float Lf[36], bool& noise);
void mp_step_launches(mp_filter f, bool pred, const float dq[7], const float L[36], bool noise, hipStream_t s);

// residual field outside the gate: d_max / sqrt(eps + sigma_s^2), the largest r inside it
inline float mp_residual_r_out(float d_max, float sigma_s, float eps) {
    return (float)((double)d_max / __builtin_sqrt((double)eps + (double)sigma_s * (double)sigma_s));
}

// surrogate (surrogate.hip)
void mp_sur_alloc(mp_surrogate S, hipStream_t s);
void mp_sur_init_weights(mp_surrogate S, hipStream_t s);
void mp_sur_reset_adam(mp_surrogate S, hipStream_t s);
void mp_sur_publish(mp_surrogate S, hipStream_t s);
void mp_sur_label(mp_surrogate S, const float* xyz_dev, int64_t n, float* out4_dev, bool scaled, hipStream_t s);
void mp_sur_eval(mp_surrogate S, const float* xyz_dev, int64_t n, float* out4_dev, hipStream_t s);
// mean |min(r_net^2, c_max) - min(r^2, c_max)| over the scan points transformed
// by every pstride-th particle (synchronises the stream)
float mp_sur_check(mp_filter f, int32_t pstride, hipStream_t s);
void mp_sur_ensure_batch(mp_surrogate S, int64_t cap);
void mp_sur_grad_step(mp_surrogate S, int32_t n_real, bool update, float lr, float* loss_dev, hipStream_t s);
// one Adam step on a batch drawn from the training set (step counter `step`)
void mp_sur_train_step(mp_surrogate S, int32_t n_real, bool full, uint32_t step, float lr, float* loss_dev,
                       hipStream_t s);
void mp_sur_likelihood(mp_filter f, float* partial, hipStream_t s);
