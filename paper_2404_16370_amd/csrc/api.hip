// api.hip -- the C-ABI of libmegapf: argument validation, handle lifetime,
// host/device pointer staging, the filter-step schedule and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <numeric>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "megapf.h"
#include "mp_internal.hpp"

// ------------------------------------------------------------ errors
static thread_local std::string g_err;

void mp_throw(mp_status code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw MpError{code, std::string(buf)};
}

template <class F>
static mp_status guarded(const char* where, F&& fn) {
    try {
        fn();
        return MP_OK;
    } catch (const MpError& e) {
        g_err = std::string(where) + ": " + e.msg;
        return e.code;
    } catch (const std::exception& e) {
        g_err = std::string(where) + ": " + e.what();
        return MP_E_HIP;
    }
}

extern "C" const char* mp_last_error(void) { return g_err.c_str(); }

// error handling of the other translation units' entry points
mp_status mp_guarded_call(const char* where, void (*fn)(void*), void* ctx) {
    return guarded(where, [&]() { fn(ctx); });
}

// ------------------------------------------------------------ device memory
void DevMem::alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    const hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        mp_throw(e == hipErrorOutOfMemory ? MP_E_OOM : MP_E_HIP, "hipMalloc(%zu): %s", b, hipGetErrorString(e));
    }
    bytes = b;
}
void DevMem::ensure(size_t b) {
    if (bytes < b) alloc(b);
}
void DevMem::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

static inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

static bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// bring `bytes` of caller data into device memory (no copy for device pointers)
static const void* stage_in(const void* src, size_t bytes, DevMem& tmp, hipStream_t s) {
    if (bytes == 0) return nullptr;
    if (is_device_ptr(src)) return src;
    tmp.ensure(bytes);
    MP_HIP(hipMemcpyAsync(tmp.p, src, bytes, hipMemcpyHostToDevice, s));
    return tmp.p;
}

// copy caller data to host memory (for validation)
static void fetch_host(const void* src, size_t bytes, void* dst, hipStream_t s) {
    if (bytes == 0) return;
    if (is_device_ptr(src)) {
        MP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
    } else {
        std::memcpy(dst, src, bytes);
    }
}

static void copy_out(void* dst, const void* src_dev, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    MP_HIP(hipMemcpyAsync(dst, src_dev, bytes, hipMemcpyDefault, s));
    if (!is_device_ptr(dst)) MP_HIP(hipStreamSynchronize(s));
}

static bool all_finite(const float* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ------------------------------------------------------------ map
extern "C" void mp_map_default_params(mp_map_params* p) {
    if (!p) return;
    p->voxel = 0.5f;
    p->nnf_radius = 2;
    p->min_points = 5;
    p->cov_eps = 1e-3f;
    p->backend = MP_NNF_AUTO;
    p->gauss_mode = MP_GAUSS_VOXEL;
    p->point_k = 10;
    p->point_search = 2;
}

extern "C" mp_status mp_map_build(const float* xyz, int64_t n, const mp_map_params* params, void* stream,
                                  mp_map* out) {
    return guarded("mp_map_build", [&]() {
        if (!out || !params || n < 0 || (n > 0 && !xyz)) mp_throw(MP_E_ARG, "null argument or n < 0");
        if (!(params->voxel > 0.0f) || !std::isfinite(params->voxel)) mp_throw(MP_E_ARG, "voxel must be > 0");
        if (params->nnf_radius < 0 || params->nnf_radius > 8) mp_throw(MP_E_ARG, "nnf_radius must be 0..8");
        if (params->min_points < 3) mp_throw(MP_E_ARG, "min_points must be >= 3");
        if (!(params->cov_eps > 0.0f && params->cov_eps <= 1.0f)) mp_throw(MP_E_ARG, "cov_eps must be in (0, 1]");
        if (params->backend < MP_NNF_AUTO || params->backend > MP_NNF_DENSE) mp_throw(MP_E_ARG, "bad backend");
        if (params->gauss_mode != MP_GAUSS_VOXEL && params->gauss_mode != MP_GAUSS_POINT)
            mp_throw(MP_E_ARG, "bad gauss_mode");
        if (params->gauss_mode == MP_GAUSS_POINT) {
            if (params->point_k < 3 || params->point_k > 32) mp_throw(MP_E_ARG, "point_k must be 3..32");
            if (params->point_search < 1 || params->point_search > 4) mp_throw(MP_E_ARG, "point_search must be 1..4");
            if (params->nnf_radius < 1)
                mp_throw(MP_E_ARG, "per-point Gaussians need nnf_radius >= 1 (the field reaches nnf_radius * voxel)");
            if (params->backend == MP_NNF_HASH)
                mp_throw(MP_E_UNSUPPORTED, "per-point Gaussians take the dense field only");
        }
        if (n > (int64_t)INT32_MAX) mp_throw(MP_E_UNSUPPORTED, "more than 2^31-1 map points");
        hipStream_t s = as_stream(stream);
        mp_map m = new mp_map_s();
        m->params = *params;
        try {
            DevMem tmp;
            const float* d = static_cast<const float*>(stage_in(xyz, sizeof(float) * 3 * (size_t)n, tmp, s));
            mp_build_map(m, d, n, s);
            MP_HIP(hipStreamSynchronize(s));
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

extern "C" mp_status mp_debug_map_point_knn(const float* xyz, int64_t n, const mp_map_params* params,
                                            int32_t* knn_out, void* stream) {
    return guarded("mp_debug_map_point_knn", [&]() {
        if (!params || !knn_out || n <= 0 || !xyz) mp_throw(MP_E_ARG, "null argument or n <= 0");
        if (params->gauss_mode != MP_GAUSS_POINT) mp_throw(MP_E_ARG, "gauss_mode must be POINT");
        if (params->point_k < 3 || params->point_k > 32) mp_throw(MP_E_ARG, "point_k must be 3..32");
        if (n > (int64_t)INT32_MAX) mp_throw(MP_E_UNSUPPORTED, "more than 2^31-1 map points");
        hipStream_t s = as_stream(stream);
        const size_t bytes = sizeof(int32_t) * (size_t)n * (size_t)params->point_k;
        DevMem lists;
        lists.alloc(bytes);
        mp_map m = new mp_map_s();
        m->params = *params;
        m->knn_dbg = lists.as<int32_t>();
        try {
            DevMem tmp;
            const float* d = static_cast<const float*>(stage_in(xyz, sizeof(float) * 3 * (size_t)n, tmp, s));
            mp_build_map(m, d, n, s);
            MP_HIP(hipMemcpyAsync(knn_out, lists.p, bytes, hipMemcpyDefault, s));
            MP_HIP(hipStreamSynchronize(s));
        } catch (...) {
            delete m;
            throw;
        }
        delete m;
    });
}

namespace {
__global__ void k_iota(int32_t* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}
}  // namespace

extern "C" mp_status mp_debug_sort_u32(const uint32_t* keys, int64_t n, int32_t bits, uint32_t* keys_out,
                                       int32_t* order_out, void* stream) {
    return guarded("mp_debug_sort_u32", [&]() {
        if (!keys || !keys_out || !order_out || n <= 0) mp_throw(MP_E_ARG, "null argument or n <= 0");
        if (bits < 1 || bits > 32) mp_throw(MP_E_ARG, "bits must be 1..32");
        if (n >= ((int64_t)1 << 30)) mp_throw(MP_E_UNSUPPORTED, "2^30 or more keys");
        hipStream_t s = as_stream(stream);
        DevMem k, k2, v, v2, scratch;
        k.alloc(sizeof(uint32_t) * (size_t)n);
        k2.alloc(sizeof(uint32_t) * (size_t)n);
        v.alloc(sizeof(int32_t) * (size_t)n);
        v2.alloc(sizeof(int32_t) * (size_t)n);
        scratch.alloc(mp_radix_scratch_bytes(n));
        mp_fill_u32(mp_radix_wait_flag(scratch), 0u, 1, s);
        MP_HIP(hipMemcpyAsync(k.p, keys, sizeof(uint32_t) * (size_t)n, hipMemcpyDefault, s));
        k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(v.as<int32_t>(), n);
        MP_CHECK_LAUNCH();
        mp_radix_sort_u32(k.as<uint32_t>(), v.as<int32_t>(), k2.as<uint32_t>(), v2.as<int32_t>(), n, bits, scratch, s);
        uint32_t waited = 0;
        MP_HIP(hipMemcpyAsync(keys_out, k.p, sizeof(uint32_t) * (size_t)n, hipMemcpyDefault, s));
        MP_HIP(hipMemcpyAsync(order_out, v.p, sizeof(int32_t) * (size_t)n, hipMemcpyDefault, s));
        MP_HIP(hipMemcpyAsync(&waited, mp_radix_wait_flag(scratch), 4, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        if (waited == 1) mp_throw(MP_E_HIP, "a sort workgroup stopped waiting for its predecessors' digit counts");
        if (waited) mp_throw(MP_E_HIP, "a key's sorted place fell outside the output");
    });
}

extern "C" mp_status mp_map_get_info(mp_map map, mp_map_info* out) {
    return guarded("mp_map_get_info", [&]() {
        if (!map || !out) mp_throw(MP_E_ARG, "null argument");
        *out = map->info;
    });
}

extern "C" mp_status mp_map_get_gauss(mp_map map, float* mu, float* normal, int32_t* voxel, int32_t* count,
                                      void* stream) {
    return guarded("mp_map_get_gauss", [&]() {
        if (!map) mp_throw(MP_E_ARG, "null map");
        const int64_t G = map->info.num_gauss;
        if (G == 0) return;
        hipStream_t s = as_stream(stream);
        std::vector<float4> g((size_t)(2 * G));
        MP_HIP(hipMemcpyAsync(g.data(), map->gauss.p, sizeof(float4) * 2 * G, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        std::vector<float> hm(3 * G), hn(3 * G);
        std::vector<int32_t> hv(3 * G), hc(G);
        MP_HIP(hipMemcpyAsync(hv.data(), map->vox.p, sizeof(int32_t) * 3 * G, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        for (int64_t k = 0; k < G; ++k) {
            hm[3 * k] = g[2 * k].x; hm[3 * k + 1] = g[2 * k].y; hm[3 * k + 2] = g[2 * k].z;
            hc[k] = (int32_t)g[2 * k].w;
            hn[3 * k] = g[2 * k + 1].x; hn[3 * k + 1] = g[2 * k + 1].y; hn[3 * k + 2] = g[2 * k + 1].z;
        }
        if (mu) copy_out(mu, hm.data(), sizeof(float) * 3 * G, s);
        if (normal) copy_out(normal, hn.data(), sizeof(float) * 3 * G, s);
        if (voxel) copy_out(voxel, hv.data(), sizeof(int32_t) * 3 * G, s);
        if (count) copy_out(count, hc.data(), sizeof(int32_t) * G, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_map_lookup(mp_map map, const float* xyz, int64_t n, int32_t* gid_out, void* stream) {
    return guarded("mp_map_lookup", [&]() {
        if (!map || n < 0 || (n > 0 && (!xyz || !gid_out))) mp_throw(MP_E_ARG, "null argument or n < 0");
        if (n == 0) return;
        hipStream_t s = as_stream(stream);
        DevMem tin, tout;
        const float* d = static_cast<const float*>(stage_in(xyz, sizeof(float) * 3 * (size_t)n, tin, s));
        if (map->info.num_gauss == 0) {
            std::vector<int32_t> miss((size_t)n, -1);
            copy_out(gid_out, miss.data(), sizeof(int32_t) * n, s);
            MP_HIP(hipStreamSynchronize(s));
            return;
        }
        int32_t* o = gid_out;
        const bool dev_out = is_device_ptr(gid_out);
        if (!dev_out) {
            tout.alloc(sizeof(int32_t) * (size_t)n);
            o = tout.as<int32_t>();
        }
        mp_map_lookup_launch(map->view, d, n, o, s);
        if (!dev_out) copy_out(gid_out, o, sizeof(int32_t) * n, s);
    });
}

extern "C" mp_status mp_map_destroy(mp_map map) {
    return guarded("mp_map_destroy", [&]() {
        if (!map) return;
        if (map->users > 0) mp_throw(MP_E_STATE, "map still used by %d filter(s)", map->users);
        MP_HIP(hipDeviceSynchronize());
        delete map;
    });
}

// ------------------------------------------------------------ filter
extern "C" void mp_filter_default_params(mp_filter_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_particles = 4096;
    p->k = 16;
    p->lsh_bits = 20;
    p->svgd_iters = 10;
    p->post_iters = 10;
    p->window_c = 32;
    p->scan_k = 10;
    p->sigma_r = 5.0f;
    p->sigma_t = 2.5f;
    p->lsh_alpha = 1.0f;
    p->lsh_sigma = 0.3f;
    p->c_max = 9.0f;
    p->d_max = 1.0f;
    p->lambda_rel = 1e-3f;
    p->lambda_abs = 1e-6f;
    p->temperature = 1.0f;
    p->prior_floor = 1e-30f;
    p->cov_eps = 1e-3f;
    p->lik_chunks = 0;
    p->lik_batch = 0;
    p->scorer = MP_SCORER_PLAIN;
    p->sigma_s = 0.03f;
    p->lsh_tangent = MP_LSH_TANGENT_DECOUPLED;
    p->lsh_tables = 1;
    p->svgd_grad = MP_SVGD_GRAD_APPROX;
    p->svgd_transport = MP_SVGD_TRANSPORT_NONE;
    p->final_rescore = 0;
    p->seed = 1;
}

static void validate_params(const mp_filter_params& p) {
    if (p.n_particles < 1 || p.n_particles > (1 << 26)) mp_throw(MP_E_ARG, "n_particles must be 1..2^26");
    if (p.k < 1 || p.k > 32) mp_throw(MP_E_ARG, "k must be 1..32");
    if (p.lsh_bits < 0 || p.lsh_bits > 30) mp_throw(MP_E_ARG, "lsh_bits must be 0..30");
    if (p.svgd_iters < 0 || p.post_iters < 0 || p.window_c < 0) mp_throw(MP_E_ARG, "negative iteration count");
    if (p.scan_k < 3 || p.scan_k > 32) mp_throw(MP_E_ARG, "scan_k must be 3..32");
    const float fs[] = {p.sigma_r, p.sigma_t, p.lsh_alpha, p.lsh_sigma, p.c_max, p.d_max,
                        p.lambda_rel, p.lambda_abs, p.temperature, p.prior_floor, p.cov_eps};
    for (float v : fs)
        if (!std::isfinite(v)) mp_throw(MP_E_ARG, "non-finite parameter");
    if (p.sigma_r < 0 || p.sigma_t < 0 || p.lsh_alpha <= 0 || p.lsh_sigma < 0 || p.c_max <= 0 || p.d_max <= 0 ||
        p.lambda_rel < 0 || p.lambda_abs < 0 || p.temperature <= 0 || p.prior_floor < 0 || p.cov_eps <= 0 ||
        p.cov_eps > 1)
        mp_throw(MP_E_ARG, "parameter out of range");
    if (p.lik_chunks < 0) mp_throw(MP_E_ARG, "lik_chunks must be >= 0");
    if (p.lik_batch != 0 && p.lik_batch != 1 && p.lik_batch != 2 && p.lik_batch != 4 && p.lik_batch != 8 &&
        p.lik_batch != 16 && p.lik_batch != 32)
        mp_throw(MP_E_ARG, "lik_batch must be 0, 1, 2, 4, 8, 16 or 32");
    if (p.scorer < MP_SCORER_PLAIN || p.scorer > MP_SCORER_SURROGATE) mp_throw(MP_E_ARG, "unknown scorer");
    if (p.lik_layout < MP_LIK_LAYOUT_AUTO || p.lik_layout > MP_LIK_LAYOUT_GROUPED) mp_throw(MP_E_ARG, "unknown lik_layout");
    if (!std::isfinite(p.sigma_s) || !(p.sigma_s > 0.0f)) mp_throw(MP_E_ARG, "sigma_s must be positive");
    if (p.lsh_tangent != MP_LSH_TANGENT_DECOUPLED && p.lsh_tangent != MP_LSH_TANGENT_SE3)
        mp_throw(MP_E_ARG, "unknown lsh_tangent");
    if (p.lsh_tables < 0 || p.lsh_tables > 16) mp_throw(MP_E_ARG, "lsh_tables must be 0..16");
    if (p.svgd_grad != MP_SVGD_GRAD_APPROX && p.svgd_grad != MP_SVGD_GRAD_EXACT) mp_throw(MP_E_ARG, "unknown svgd_grad");
    if (p.svgd_transport != MP_SVGD_TRANSPORT_NONE && p.svgd_transport != MP_SVGD_TRANSPORT_ADJOINT)
        mp_throw(MP_E_ARG, "unknown svgd_transport");
    if (p.final_rescore != 0 && p.final_rescore != 1) mp_throw(MP_E_ARG, "final_rescore must be 0 or 1");
}

static void destroy_filter(mp_filter f) {
    if (!f) return;
    for (int st = 0; st < MP_NUM_STAGES; ++st) {
        for (hipEvent_t e : f->ev0[st]) (void)hipEventDestroy(e);
        for (hipEvent_t e : f->ev1[st]) (void)hipEventDestroy(e);
    }
    if (f->map) f->map->users--;
    if (f->sur) f->sur->users--;
    delete f;
}

extern "C" mp_status mp_filter_init(mp_map map, const mp_filter_params* params, const mp_init_desc* init,
                                    void* stream, mp_filter* out) {
    return guarded("mp_filter_init", [&]() {
        if (!map || !params || !init || !out) mp_throw(MP_E_ARG, "null argument");
        validate_params(*params);
        const int n = params->n_particles;
        hipStream_t s = as_stream(stream);
        std::vector<float> host_poses;
        float gmean[7], gL[36];
        bool gnoise = false;
        if (init->kind == MP_INIT_EXPLICIT) {
            if (!init->poses) mp_throw(MP_E_ARG, "explicit init without poses");
            std::vector<float> p7((size_t)n * 7);
            fetch_host(init->poses, sizeof(float) * 7 * (size_t)n, p7.data(), s);
            if (!all_finite(p7.data(), p7.size())) mp_throw(MP_E_ARG, "non-finite initial pose");
            host_poses.assign((size_t)n * 8, 0.0f);
            for (int i = 0; i < n; ++i) {
                const float* q = &p7[7 * (size_t)i];
                const double nq = std::sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                                            (double)q[3] * q[3]);
                if (!(nq > 1e-12)) mp_throw(MP_E_ARG, "zero quaternion for particle %d", i);
                const bool unit = std::fabs(nq - 1.0) < 1e-6;
                for (int k = 0; k < 4; ++k) host_poses[8 * (size_t)i + k] = unit ? q[k] : (float)(q[k] / nq);
                for (int k = 0; k < 3; ++k) host_poses[8 * (size_t)i + 4 + k] = q[4 + k];
            }
        } else if (init->kind == MP_INIT_UNIFORM_BOX) {
            if (!all_finite(init->box_min, 3) || !all_finite(init->box_max, 3)) mp_throw(MP_E_ARG, "non-finite box");
            for (int a = 0; a < 3; ++a)
                if (init->box_max[a] < init->box_min[a]) mp_throw(MP_E_ARG, "box_max < box_min");
        } else if (init->kind == MP_INIT_GAUSSIAN) {
            // the mean replicated, then moved by exp(L z_i) as a prediction from it would be
            mp_prepare_prediction(init->mean, init->cov, gmean, gL, gnoise);
            host_poses.assign((size_t)n * 8, 0.0f);
            for (int i = 0; i < n; ++i)
                for (int k = 0; k < 7; ++k) host_poses[8 * (size_t)i + k] = gmean[k];
        } else {
            mp_throw(MP_E_ARG, "unknown init kind %d", init->kind);
        }
        mp_filter f = new mp_filter_s();
        try {
            f->map = map;
            map->users++;
            f->p = *params;
            f->n = n;
            f->K = params->k;
            for (int a = 0; a < 3; ++a) {
                f->lsh_lo[a] = map->box_lo[a];
                f->lsh_hi[a] = map->box_hi[a];
            }
            const size_t N = (size_t)n, K = (size_t)params->k;
            f->poses[0].alloc(32 * N);
            f->poses[1].alloc(32 * N);
            f->psi.alloc(32 * N);
            f->codes.alloc(4 * N);
            f->sorted.alloc(4 * N);
            f->scodes.alloc(4 * N);
            f->tmp_keys.alloc(4 * N);
            f->tmp_vals.alloc(4 * N);
            f->lkeys.alloc(4 * N);
            f->lorder.alloc(4 * N);
            f->head.alloc(4 * N);
            f->end.alloc(4 * N);
            f->rank.alloc(4 * N);
            f->hist.alloc(mp_radix_scratch_bytes(n));
            f->nbr.alloc(4 * K * N);
            f->kval.alloc(4 * K * N);
            f->cnt.alloc(4 * N);
            f->prior.alloc(4 * N);
            f->post0.alloc(4 * N);
            f->post1.alloc(4 * N);
            f->flags.alloc(64);
            f->tlsh.alloc(32);
            f->stepinfo.alloc(16 * sizeof(double));
            f->red.alloc(sizeof(double) * (N + 3 * ((N + 255) / 256)) + sizeof(int) * ((N + 255) / 256) + 64);
            MP_HIP(hipMemsetAsync(f->flags.p, 0, 64, s));
            MP_HIP(hipMemsetAsync(f->stepinfo.p, 0, 16 * sizeof(double), s));
            MP_HIP(hipMemsetAsync(f->psi.p, 0, 32 * N, s));
            MP_HIP(hipMemsetAsync(f->tlsh.p, 0, 32, s));
            MP_HIP(hipMemsetAsync(f->post1.p, 0, 4 * N, s));
            if (init->kind == MP_INIT_EXPLICIT || init->kind == MP_INIT_GAUSSIAN) {
                MP_HIP(hipMemcpyAsync(f->poses[0].p, host_poses.data(), 32 * N, hipMemcpyHostToDevice, s));
                if (init->kind == MP_INIT_GAUSSIAN) {
                    static const float ident[7] = {1, 0, 0, 0, 0, 0, 0};
                    mp_launch_predict(f, ident, gL, gnoise, s, true);
                }
                MP_HIP(hipStreamSynchronize(s));
            } else {
                mp_launch_init_uniform(f, init->box_min, init->box_max, s);
            }
            mp_launch_reset_lists(f, s);
        } catch (...) {
            destroy_filter(f);
            throw;
        }
        *out = f;
    });
}

extern "C" mp_status mp_filter_destroy(mp_filter f) {
    return guarded("mp_filter_destroy", [&]() {
        if (!f) return;
        if (f->batch_users > 0) mp_throw(MP_E_STATE, "filter still held by %d batch(es)", f->batch_users);
        MP_HIP(hipDeviceSynchronize());
        destroy_filter(f);
    });
}

extern "C" mp_status mp_scan_upload(mp_filter f, const float* xyz, const float* cov6, int32_t n, void* stream) {
    return guarded("mp_scan_upload", [&]() {
        if (!f || n < 0 || (n > 0 && !xyz)) mp_throw(MP_E_ARG, "null argument or n < 0");
        if (n > 65536) mp_throw(MP_E_ARG, "more than 65536 scan points");
        hipStream_t s = as_stream(stream);
        if (n > 0) {
            f->scan_xyz.ensure(sizeof(float) * 3 * (size_t)n);
            f->scan.ensure(sizeof(float) * 12 * (size_t)n);
            f->scan_perm.ensure(sizeof(int32_t) * (size_t)n);
            f->scan_work.ensure(sizeof(uint32_t) * (4 * (size_t)n + 4));
            f->scan_sort.ensure(mp_radix_scratch_bytes(n));
            // caller data (host or device) into the filter's staging buffers
            MP_HIP(hipMemcpyAsync(f->scan_xyz.p, xyz, sizeof(float) * 3 * (size_t)n, hipMemcpyDefault, s));
            const float* dcov = nullptr;
            if (cov6) {
                f->scan_cov.ensure(sizeof(float) * 6 * (size_t)n);
                MP_HIP(hipMemcpyAsync(f->scan_cov.p, cov6, sizeof(float) * 6 * (size_t)n, hipMemcpyDefault, s));
                dcov = f->scan_cov.as<float>();
            }
            uint32_t* work = f->scan_work.as<uint32_t>();
            float* lo_bad = reinterpret_cast<float*>(work + 4 * (size_t)n);
            // validation on the device; only its 4-byte verdict comes back
            mp_scan_check(f->scan_xyz.as<float>(), dcov, n, lo_bad, s);
            float bad = 0.0f;
            MP_HIP(hipMemcpyAsync(&bad, lo_bad + 3, sizeof(float), hipMemcpyDeviceToHost, s));
            MP_HIP(hipStreamSynchronize(s));
            if (bad != 0.0f) mp_throw(MP_E_ARG, cov6 ? "non-finite scan point or covariance" : "non-finite scan point");
            // the current records become the previous scan's (odometry)
            if (f->orig_n > 0) {
                f->scan_orig.swap(f->prev_orig);
                f->prev_n = f->orig_n;
            }
            f->scan_orig.ensure(sizeof(float) * 12 * (size_t)n);
            f->orig_n = n;
            f->ev_count[MP_STAGE_SCAN] = 0;
            mp_tick(f, MP_STAGE_SCAN, true, s);
            // Walk order for the likelihood: Morton order of the points on a grid of half the
            // map voxel, so that consecutive points of one particle land in the same or
            // neighbouring voxels (the sum over points does not depend on the order).
            mp_scan_walk_order(f->scan_xyz.as<float>(), n, 0.5f * f->map->params.voxel, lo_bad, work, work + n,
                               f->scan_perm.as<int32_t>(), reinterpret_cast<int32_t*>(work + 2 * (size_t)n),
                               f->scan_sort, s);
            mp_scan_records(f->scan_xyz.as<float>(), dcov, n, f->p.scan_k, f->p.cov_eps, f->scan_orig.as<float>(), s);
            mp_scan_permute(f->scan_orig.as<float>(), f->scan_perm.as<int32_t>(), n, f->scan.as<float>(), s);
            mp_tick(f, MP_STAGE_SCAN, false, s);
        }
        f->scan_n = n;
        f->last_stream = s;
    });
}

void mp_tick(mp_filter f, int st, bool begin, hipStream_t s) {
    if (f->capturing) return;
    const int k = f->ev_count[st];
    auto& v = begin ? f->ev0[st] : f->ev1[st];
    while ((int)v.size() <= k) {
        hipEvent_t e;
        MP_HIP(hipEventCreate(&e));
        v.push_back(e);
    }
    MP_HIP(hipEventRecord(v[k], s));
    if (!begin) f->ev_count[st] = k + 1;
}

// host FP64 Cholesky of a 6x6 PSD matrix; false if not PSD
static bool chol6_host(const double A[36], double L[36]) {
    std::memset(L, 0, sizeof(double) * 36);
    double scale = 0.0;
    for (int i = 0; i < 6; ++i) scale = std::fmax(scale, std::fabs(A[7 * i]));
    const double tol = -1e-9 * (scale > 0 ? scale : 1.0);
    for (int j = 0; j < 6; ++j) {
        double s = A[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (s < tol) return false;
        s = s > 0 ? s : 0.0;
        L[6 * j + j] = std::sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = A[6 * i + j];
            for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = L[6 * j + j] > 0 ? t / L[6 * j + j] : 0.0;
        }
    }
    return true;
}

void mp_prepare_prediction(const float dT[7], const float cov[36], float dq[7], float Lf[36], bool& noise) {
    if (!all_finite(dT, 7)) mp_throw(MP_E_ARG, "non-finite dT");
    const double nq = std::sqrt((double)dT[0] * dT[0] + (double)dT[1] * dT[1] + (double)dT[2] * dT[2] +
                                (double)dT[3] * dT[3]);
    if (!(nq > 1e-12)) mp_throw(MP_E_ARG, "zero quaternion in dT");
    for (int k = 0; k < 4; ++k) dq[k] = (float)(dT[k] / nq);
    for (int k = 0; k < 3; ++k) dq[4 + k] = dT[4 + k];
    noise = false;
    std::memset(Lf, 0, sizeof(float) * 36);
    if (cov) {
        if (!all_finite(cov, 36)) mp_throw(MP_E_ARG, "non-finite cov_dT");
        double A[36], L[36];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                if (std::fabs((double)cov[6 * i + j] - (double)cov[6 * j + i]) >
                    1e-6 * (1.0 + std::fabs((double)cov[6 * i + j])))
                    mp_throw(MP_E_ARG, "cov_dT not symmetric");
                A[6 * i + j] = cov[6 * i + j];
            }
        if (!chol6_host(A, L)) mp_throw(MP_E_ARG, "cov_dT not positive semi-definite");
        for (int k = 0; k < 36; ++k) Lf[k] = (float)L[k];
        noise = true;
    }
}

static void run_stage(mp_filter f, int st, int it, hipStream_t s) {
    switch (st) {
        case MP_STAGE_LSH: mp_launch_lsh(f, (uint32_t)f->frame, (uint32_t)it, s); break;
        case MP_STAGE_SORT: mp_launch_sort(f, s); break;
        case MP_STAGE_REFRESH: mp_launch_refresh(f, s); break;
        case MP_STAGE_LIK: mp_launch_likelihood(f, s); break;
        case MP_STAGE_SVGD: mp_launch_svgd(f, s); break;
        case MP_STAGE_POSTERIOR: mp_launch_posterior(f, s); break;
        default: mp_throw(MP_E_ARG, "stage %d cannot run alone", st);
    }
}

// the likelihood and the lists' kernel values at the current (final) poses:
// one likelihood pass and a refresh that only re-ranks the current lists
static void rescore(mp_filter f, hipStream_t s) {
    mp_tick(f, MP_STAGE_LIK, true, s);
    run_stage(f, MP_STAGE_LIK, f->p.svgd_iters, s);
    mp_tick(f, MP_STAGE_LIK, false, s);
    mp_tick(f, MP_STAGE_REFRESH, true, s);
    mp_launch_refresh(f, s, 0);
    mp_tick(f, MP_STAGE_REFRESH, false, s);
}

void mp_reserve_step(mp_filter f) {
    f->partial.ensure(mp_lik_partial_bytes(f));
    f->red.ensure(std::max(mp_post_scratch_bytes(f), sizeof(uint32_t) * ((size_t)f->n + 64)));
    f->hist.ensure(mp_radix_scratch_bytes(f->n));
}

void mp_step_begin(mp_filter f, bool pred, const float dq[7], const float L[36], bool noise, hipStream_t s) {
    mp_fill_u32(f->flags.p, 0u, 4, s);
    // a captured step always holds the prediction node; it reads whether to
    // predict from the step values
    if (pred || f->dyn) {
        static const float ident[7] = {1, 0, 0, 0, 0, 0, 0};
        static const float zero[36] = {};
        mp_tick(f, MP_STAGE_PREDICT, true, s);
        mp_launch_predict(f, pred ? dq : ident, pred ? L : zero, pred && noise, s);
        mp_tick(f, MP_STAGE_PREDICT, false, s);
    }
}

// per iteration, in the order of Table II: neighbour list update (LSH, sort,
// refresh; once per hash table, table l of iteration it drawing with counter
// it * tables + l), likelihood evaluation, particle state update
void mp_step_iter_nbr(mp_filter f, int it, hipStream_t s) {
    const int tables = std::max(1, f->p.lsh_tables);
    for (int l = 0; l < tables; ++l)
        for (int st : {MP_STAGE_LSH, MP_STAGE_SORT, MP_STAGE_REFRESH}) {
            mp_tick(f, st, true, s);
            run_stage(f, st, it * tables + l, s);
            mp_tick(f, st, false, s);
        }
}

void mp_step_iter_svgd(mp_filter f, int it, hipStream_t s) {
    mp_tick(f, MP_STAGE_SVGD, true, s);
    run_stage(f, MP_STAGE_SVGD, it, s);
    mp_tick(f, MP_STAGE_SVGD, false, s);
}

void mp_step_end(mp_filter f, hipStream_t s) {
    if (f->scan_n <= 0 || f->p.svgd_iters <= 0) return;
    if (f->p.final_rescore) rescore(f, s);
    mp_tick(f, MP_STAGE_POSTERIOR, true, s);
    mp_launch_posterior(f, s);
    mp_tick(f, MP_STAGE_POSTERIOR, false, s);
}

void mp_step_launches(mp_filter f, bool pred, const float dq[7], const float L[36], bool noise, hipStream_t s) {
    mp_step_begin(f, pred, dq, L, noise, s);
    if (f->scan_n > 0) {
        for (int it = 0; it < f->p.svgd_iters; ++it) {
            mp_step_iter_nbr(f, it, s);
            mp_tick(f, MP_STAGE_LIK, true, s);
            run_stage(f, MP_STAGE_LIK, it, s);
            mp_tick(f, MP_STAGE_LIK, false, s);
            mp_step_iter_svgd(f, it, s);
        }
    }
    mp_step_end(f, s);
}

extern "C" mp_status mp_filter_step(mp_filter f, const float dT[7], const float cov_dT[36], void* stream) {
    return guarded("mp_filter_step", [&]() {
        if (!f) mp_throw(MP_E_ARG, "null filter");
        if (f->scan_n < 0) mp_throw(MP_E_STATE, "mp_filter_step before the first mp_scan_upload");
        if (f->p.scorer == MP_SCORER_SURROGATE && !f->sur)
            mp_throw(MP_E_STATE, "SURROGATE scorer without a network (mp_filter_set_surrogate)");
        hipStream_t s = as_stream(stream);
        float dq[7], L[36];
        bool noise = false;
        if (dT) mp_prepare_prediction(dT, cov_dT, dq, L, noise);
        // every work buffer of the step is sized before anything is launched,
        // so that a failed allocation leaves the filter as it was
        mp_reserve_step(f);
        for (int st = 0; st < MP_NUM_STAGES; ++st)
            if (st != MP_STAGE_SCAN) f->ev_count[st] = 0;
        // check of the learned scorer (before the step, on the current particles)
        f->sur_fallback = false;
        SurCheck& c = f->chk;
        if (f->p.scorer == MP_SCORER_SURROGATE && c.period > 0 && f->scan_n > 0) {
            if (c.left == 0 && f->frame % c.period == 0) {
                c.last = mp_sur_check(f, c.stride, s);
                ++c.checks;
                if (!(c.last <= c.threshold)) c.left = c.fallback;
            }
            if (c.left > 0) {
                f->sur_fallback = true;
                --c.left;
                ++c.fallback_steps;
            }
        }
        mp_step_launches(f, dT != nullptr, dq, L, noise, s);
        f->sur_fallback = false;
        f->frame++;
        f->last_stream = s;
    });
}

extern "C" mp_status mp_posterior_query(mp_filter f, mp_posterior* out, float* poses_out, double* weights_out,
                                        void* stream) {
    return guarded("mp_posterior_query", [&]() {
        if (!f || !out) mp_throw(MP_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        double info[16];
        int32_t flags[16];
        MP_HIP(hipMemcpyAsync(info, f->stepinfo.p, sizeof(info), hipMemcpyDeviceToHost, s));
        MP_HIP(hipMemcpyAsync(flags, f->flags.p, sizeof(flags), hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        int idx = (int)info[7];
        if (idx < 0 || idx >= f->n) idx = 0;
        float pose[8];
        MP_HIP(hipMemcpyAsync(pose, f->poses[f->cur].as<float>() + 8 * (size_t)idx, 32, hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
        std::memset(out, 0, sizeof(*out));
        for (int k = 0; k < 7; ++k) out->map_pose[k] = pose[k];
        out->map_index = idx;
        out->map_weight = info[4];
        out->n_eff = info[5];
        out->log_evidence = info[2];
        out->max_loglik = info[6];
        out->frame = f->frame;
        out->fp64_resolves = flags[0];
        out->fallback_steps = f->chk.fallback_steps;
        out->sur_checks = f->chk.checks;
        out->sur_check_ds = f->chk.last;
        bool finite = all_finite(pose, 7) && std::isfinite(info[4]);
        const size_t N = (size_t)f->n;
        if (poses_out) {
            std::vector<float> p8(8 * N), p7(7 * N);
            MP_HIP(hipMemcpyAsync(p8.data(), f->poses[f->cur].p, 32 * N, hipMemcpyDeviceToHost, s));
            MP_HIP(hipStreamSynchronize(s));
            for (size_t i = 0; i < N; ++i)
                for (int k = 0; k < 7; ++k) p7[7 * i + k] = p8[8 * i + k];
            finite = finite && all_finite(p7.data(), p7.size());
            copy_out(poses_out, p7.data(), sizeof(float) * 7 * N, s);
        }
        if (weights_out) {
            std::vector<float> w(N);
            std::vector<double> wd(N);
            MP_HIP(hipMemcpyAsync(w.data(), f->prior.p, 4 * N, hipMemcpyDeviceToHost, s));
            MP_HIP(hipStreamSynchronize(s));
            for (size_t i = 0; i < N; ++i) wd[i] = w[i];
            finite = finite && all_finite(w.data(), N);
            copy_out(weights_out, wd.data(), sizeof(double) * N, s);
        }
        MP_HIP(hipStreamSynchronize(s));
        if (!finite) mp_throw(MP_E_NUMERIC, "non-finite pose or weight in the filter state");
    });
}

extern "C" mp_status mp_stage_times(mp_filter f, float* ms_out, int32_t* counts_out) {
    return guarded("mp_stage_times", [&]() {
        if (!f || !ms_out) mp_throw(MP_E_ARG, "null argument");
        for (int st = 0; st < MP_NUM_STAGES; ++st) {
            double tot = 0.0;
            for (int k = 0; k < f->ev_count[st]; ++k) {
                MP_HIP(hipEventSynchronize(f->ev1[st][k]));
                float ms = 0.0f;
                MP_HIP(hipEventElapsedTime(&ms, f->ev0[st][k], f->ev1[st][k]));
                tot += ms;
            }
            ms_out[st] = (float)tot;
            if (counts_out) counts_out[st] = f->ev_count[st];
        }
    });
}

// ------------------------------------------------------------ debug access
struct NamedBuf {
    void* p;
    size_t bytes;
    bool settable;
};

static NamedBuf lookup_buf(mp_filter f, const char* name) {
    const size_t N = (size_t)f->n, K = (size_t)f->K;
    const std::string s(name ? name : "");
    if (s == "poses") return {f->poses[f->cur].p, 32 * N, true};
    if (s == "psi") return {f->psi.p, 32 * N, true};
    if (s == "hb") {
        f->hb.ensure(28 * 4 * N);
        return {f->hb.p, 28 * 4 * N, false};
    }
    if (s == "solve") {
        f->solve_how.ensure(4 * N);
        return {f->solve_how.p, 4 * N, false};
    }
    if (s == "codes") return {f->codes.p, 4 * N, true};
    if (s == "sorted") return {f->sorted.p, 4 * N, true};
    if (s == "scodes") return {f->scodes.p, 4 * N, true};
    if (s == "head") return {f->head.p, 4 * N, true};
    if (s == "end") return {f->end.p, 4 * N, true};
    if (s == "nbr") return {f->nbr.p, 4 * K * N, true};
    if (s == "kval") return {f->kval.p, 4 * K * N, true};
    if (s == "cnt") return {f->cnt.p, 4 * N, true};
    if (s == "prior") return {f->prior.p, 4 * N, true};
    if (s == "post") return {f->prior.p, 4 * N, false};
    if (s == "post0") return {f->post0.p, 4 * N, false};
    if (s == "scan") return {f->scan_orig.p, f->scan_n > 0 ? 48 * (size_t)f->scan_n : 0, false};
    if (s == "scan_walk") return {f->scan.p, f->scan_n > 0 ? 48 * (size_t)f->scan_n : 0, false};
    if (s == "odo_nn") return {f->odo_nn.p, f->odo_nn.p && f->scan_n > 0 ? 4 * (size_t)f->scan_n : 0, false};
    if (s == "tlsh") return {f->tlsh.p, 32, false};
    if (s == "sort_wait") return {f->hist.p ? (void*)mp_radix_wait_flag(f->hist) : nullptr, f->hist.p ? 4u : 0u, false};
    mp_throw(MP_E_ARG, "unknown buffer '%s'", s.c_str());
}

extern "C" mp_status mp_debug_get(mp_filter f, const char* name, void* dst, int64_t bytes, void* stream) {
    return guarded("mp_debug_get", [&]() {
        if (!f || !dst) mp_throw(MP_E_ARG, "null argument");
        const NamedBuf b = lookup_buf(f, name);
        if ((size_t)bytes != b.bytes) mp_throw(MP_E_ARG, "'%s' holds %zu bytes, asked %lld", name, b.bytes, (long long)bytes);
        hipStream_t s = as_stream(stream);
        copy_out(dst, b.p, b.bytes, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_debug_set(mp_filter f, const char* name, const void* src, int64_t bytes, void* stream) {
    return guarded("mp_debug_set", [&]() {
        if (!f || !src) mp_throw(MP_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        if (std::string(name ? name : "") == "capture_hb") {
            if (bytes != 4) mp_throw(MP_E_ARG, "capture_hb takes one int32");
            int32_t v = 0;
            fetch_host(src, 4, &v, s);
            f->capture_hb = v ? 1 : 0;
            if (f->capture_hb) f->hb.ensure(28 * 4 * (size_t)f->n);
            if (f->capture_hb) f->solve_how.ensure(4 * (size_t)f->n);
            return;
        }
        const NamedBuf b = lookup_buf(f, name);
        if (!b.settable) mp_throw(MP_E_ARG, "'%s' is read-only", name);
        if ((size_t)bytes != b.bytes) mp_throw(MP_E_ARG, "'%s' holds %zu bytes, given %lld", name, b.bytes, (long long)bytes);
        MP_HIP(hipMemcpyAsync(b.p, src, b.bytes, hipMemcpyDefault, s));
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_debug_stage(mp_filter f, int32_t stage, int32_t iteration, const float dT[7],
                                    const float cov_dT[36], void* stream) {
    return guarded("mp_debug_stage", [&]() {
        if (!f) mp_throw(MP_E_ARG, "null filter");
        hipStream_t s = as_stream(stream);
        if (stage == MP_STAGE_PREDICT) {
            if (!dT) mp_throw(MP_E_ARG, "prediction needs dT");
            float dq[7], L[36];
            bool noise = false;
            mp_prepare_prediction(dT, cov_dT, dq, L, noise);
            mp_launch_predict(f, dq, L, noise, s);
        } else if (stage == MP_DEBUG_RESCORE) {
            if (f->scan_n < 0) mp_throw(MP_E_STATE, "no scan uploaded");
            MP_HIP(hipMemsetAsync(f->flags.p, 0, 16, s));
            rescore(f, s);
        } else {
            if ((stage == MP_STAGE_LIK) && f->scan_n < 0) mp_throw(MP_E_STATE, "no scan uploaded");
            if (stage == MP_STAGE_LIK) MP_HIP(hipMemsetAsync(f->flags.p, 0, 16, s));
            run_stage(f, stage, iteration, s);
        }
        MP_HIP(hipStreamSynchronize(s));
    });
}

// ------------------------------------------------------------ surrogate
extern "C" void mp_surrogate_default_params(mp_surrogate_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->f_max = 0.0f;
    p->sigma_s = 0.03f;
    p->d_max = 0.0f;
    p->c_max = 9.0f;
    p->lr = 1e-3f;
    p->lr_min = 1e-5f;
    p->beta1 = 0.9f;
    p->beta2 = 0.999f;
    p->adam_eps = 1e-8f;
    p->total_steps = 20000;
    p->batch = 65536;
    p->seed = 1;
}

extern "C" mp_status mp_surrogate_create(mp_map map, const mp_surrogate_params* params, void* stream,
                                         mp_surrogate* out) {
    return guarded("mp_surrogate_create", [&]() {
        if (!map || !params || !out) mp_throw(MP_E_ARG, "null argument");
        mp_surrogate_params p = *params;
        const float fs[] = {p.box_min[0], p.box_min[1], p.box_min[2], p.box_max[0], p.box_max[1], p.box_max[2],
                            p.f_max, p.sigma_s, p.d_max, p.c_max, p.lr, p.lr_min, p.beta1, p.beta2, p.adam_eps};
        for (float v : fs)
            if (!std::isfinite(v)) mp_throw(MP_E_ARG, "non-finite parameter");
        if (!(p.sigma_s > 0) || p.d_max < 0 || !(p.c_max > 0) || p.f_max < 0 || !(p.lr > 0) || p.lr_min < 0 ||
            !(p.beta1 >= 0 && p.beta1 < 1) || !(p.beta2 >= 0 && p.beta2 < 1) || !(p.adam_eps > 0) ||
            p.total_steps < 1 || p.batch < 256 || p.batch > (1 << 20))
            mp_throw(MP_E_ARG, "parameter out of range");
        const float r = map->params.voxel;
        if (p.d_max == 0.0f) p.d_max = 2.0f * r;
        bool box_given = false;
        for (int a = 0; a < 3; ++a) box_given = box_given || p.box_min[a] != p.box_max[a];
        if (!box_given) {
            if (map->info.num_gauss <= 0) mp_throw(MP_E_ARG, "empty map and no feature box");
            for (int a = 0; a < 3; ++a) {
                p.box_min[a] = map->info.box_min[a];
                p.box_max[a] = map->info.box_max[a];
            }
        }
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!(p.box_max[a] > p.box_min[a])) mp_throw(MP_E_ARG, "empty feature box");
            ext = std::max(ext, (double)p.box_max[a] - (double)p.box_min[a]);
        }
        if (p.f_max == 0.0f) p.f_max = (float)(ext / (double)r);
        if (!(p.f_max >= 1.0f)) mp_throw(MP_E_ARG, "f_max below one cycle per box");
        auto S = std::make_unique<mp_surrogate_s>();
        S->map = map;
        S->p = p;
        mp_surrogate_info& I = S->info;
        std::memset(&I, 0, sizeof(I));
        I.n_params = MP_SUR_NPARAMS;
        for (int a = 0; a < 3; ++a) {
            I.lo[a] = p.box_min[a];
            I.inv_ext[a] = (float)(1.0 / ext);
        }
        for (int l = 0; l < 32; ++l) I.freqs[l] = (float)std::pow((double)p.f_max, (double)l / 31.0);
        const double eps = map->params.cov_eps, s2 = (double)p.sigma_s * (double)p.sigma_s;
        I.r_scale = mp_residual_r_out(p.d_max, p.sigma_s, map->params.cov_eps);
        I.g_scale = (float)(1.0 / std::sqrt(eps + s2));
        I.weight_bytes = MP_SUR_IMAGE_BYTES;
        hipStream_t s = as_stream(stream);
        mp_sur_alloc(S.get(), s);
        mp_sur_init_weights(S.get(), s);
        MP_HIP(hipStreamSynchronize(s));
        map->users++;
        *out = S.release();
    });
}

extern "C" mp_status mp_surrogate_destroy(mp_surrogate sur) {
    return guarded("mp_surrogate_destroy", [&]() {
        if (!sur) return;
        if (sur->users > 0) mp_throw(MP_E_STATE, "network still used by %d filter(s)", sur->users);
        MP_HIP(hipDeviceSynchronize());
        if (sur->map) sur->map->users--;
        delete sur;
    });
}

extern "C" mp_status mp_surrogate_get_info(mp_surrogate sur, mp_surrogate_info* out) {
    return guarded("mp_surrogate_get_info", [&]() {
        if (!sur || !out) mp_throw(MP_E_ARG, "null argument");
        *out = sur->info;
    });
}

static void check_points(const float* xyz, int64_t n) {
    if (n < 0 || (n > 0 && !xyz)) mp_throw(MP_E_ARG, "bad point array");
    if (n > ((int64_t)1 << 31)) mp_throw(MP_E_ARG, "too many points");
}

extern "C" mp_status mp_surrogate_label(mp_surrogate sur, const float* xyz, int64_t n, float* out4, void* stream) {
    return guarded("mp_surrogate_label", [&]() {
        if (!sur) mp_throw(MP_E_ARG, "null surrogate");
        check_points(xyz, n);
        if (n > 0 && !out4) mp_throw(MP_E_ARG, "null output");
        if (n == 0) return;
        hipStream_t s = as_stream(stream);
        DevMem tin, tout;
        const float* d = static_cast<const float*>(stage_in(xyz, sizeof(float) * 3 * (size_t)n, tin, s));
        const bool dev_out = is_device_ptr(out4);
        float* o = out4;
        if (!dev_out) {
            tout.alloc(sizeof(float) * 4 * (size_t)n);
            o = tout.as<float>();
        }
        mp_sur_label(sur, d, n, o, false, s);
        if (!dev_out) copy_out(out4, o, sizeof(float) * 4 * (size_t)n, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_surrogate_eval(mp_surrogate sur, const float* xyz, int64_t n, float* out4, void* stream) {
    return guarded("mp_surrogate_eval", [&]() {
        if (!sur) mp_throw(MP_E_ARG, "null surrogate");
        check_points(xyz, n);
        if (n > 0 && !out4) mp_throw(MP_E_ARG, "null output");
        if (n == 0) return;
        hipStream_t s = as_stream(stream);
        DevMem tin, tout;
        const float* d = static_cast<const float*>(stage_in(xyz, sizeof(float) * 3 * (size_t)n, tin, s));
        const bool dev_out = is_device_ptr(out4);
        float* o = out4;
        if (!dev_out) {
            tout.alloc(sizeof(float) * 4 * (size_t)n);
            o = tout.as<float>();
        }
        mp_sur_eval(sur, d, n, o, s);
        if (!dev_out) copy_out(out4, o, sizeof(float) * 4 * (size_t)n, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_surrogate_set_data(mp_surrogate sur, const float* xyz, int64_t n, void* stream) {
    return guarded("mp_surrogate_set_data", [&]() {
        if (!sur) mp_throw(MP_E_ARG, "null surrogate");
        check_points(xyz, n);
        if (n < 1) mp_throw(MP_E_ARG, "training set must hold at least one point");
        hipStream_t s = as_stream(stream);
        sur->dxyz.alloc(sizeof(float) * 3 * (size_t)n);
        sur->dlab.alloc(sizeof(float) * 4 * (size_t)n);
        MP_HIP(hipMemcpyAsync(sur->dxyz.p, xyz, sizeof(float) * 3 * (size_t)n, hipMemcpyDefault, s));
        mp_sur_label(sur, sur->dxyz.as<float>(), n, sur->dlab.as<float>(), true, s);
        sur->info.n_data = n;
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_surrogate_train(mp_surrogate sur, int32_t steps, float* loss_out, void* stream) {
    return guarded("mp_surrogate_train", [&]() {
        if (!sur) mp_throw(MP_E_ARG, "null surrogate");
        if (steps < 0) mp_throw(MP_E_ARG, "negative step count");
        if (sur->info.n_data < 1) mp_throw(MP_E_STATE, "no training data (mp_surrogate_set_data)");
        if (steps == 0) return;
        hipStream_t s = as_stream(stream);
        const bool full = sur->info.n_data <= sur->p.batch;
        const int32_t n_real = full ? (int32_t)sur->info.n_data : sur->p.batch;
        mp_sur_ensure_batch(sur, n_real);
        sur->losses.ensure(sizeof(float) * (size_t)steps);
        const mp_surrogate_params& p = sur->p;
        for (int32_t k = 0; k < steps; ++k) {
            const int64_t t = sur->info.steps;   // steps taken before this one
            const double frac = std::min(1.0, (double)t / (double)p.total_steps);
            const double lr = p.lr_min + 0.5 * ((double)p.lr - p.lr_min) * (1.0 + std::cos(M_PI * frac));
            mp_sur_train_step(sur, n_real, full, (uint32_t)t, (float)lr, sur->losses.as<float>() + k, s);
        }
        if (loss_out) {
            MP_HIP(hipMemcpyAsync(loss_out, sur->losses.p, sizeof(float) * (size_t)steps, hipMemcpyDeviceToHost, s));
            MP_HIP(hipStreamSynchronize(s));
        }
    });
}

extern "C" mp_status mp_surrogate_grad(mp_surrogate sur, const float* xyz, const float* target4, int64_t n,
                                       float* grad_out, float* loss_out, void* stream) {
    return guarded("mp_surrogate_grad", [&]() {
        if (!sur || !xyz || !target4) mp_throw(MP_E_ARG, "null argument");
        if (n < 1 || n > sur->p.batch) mp_throw(MP_E_ARG, "n must be 1..batch");
        hipStream_t s = as_stream(stream);
        mp_sur_ensure_batch(sur, n);
        std::vector<float> tgt(4 * (size_t)n);
        fetch_host(target4, sizeof(float) * 4 * (size_t)n, tgt.data(), s);
        const float is = 1.0f / sur->info.r_scale, ig = 1.0f / sur->info.g_scale;
        for (int64_t i = 0; i < n; ++i) {
            tgt[4 * i] *= is;
            for (int a = 1; a < 4; ++a) tgt[4 * i + a] *= ig;
        }
        const int32_t bp = sur->cap;
        MP_HIP(hipMemsetAsync(sur->bxyz.p, 0, sizeof(float) * 3 * (size_t)bp, s));
        MP_HIP(hipMemsetAsync(sur->btgt.p, 0, sizeof(float) * 4 * (size_t)bp, s));
        MP_HIP(hipMemcpyAsync(sur->bxyz.p, xyz, sizeof(float) * 3 * (size_t)n, hipMemcpyDefault, s));
        MP_HIP(hipMemcpyAsync(sur->btgt.p, tgt.data(), sizeof(float) * 4 * (size_t)n, hipMemcpyHostToDevice, s));
        sur->losses.ensure(sizeof(float));
        mp_sur_grad_step(sur, (int32_t)n, false, 0.0f, sur->losses.as<float>(), s);
        if (grad_out) copy_out(grad_out, sur->G.p, sizeof(float) * MP_SUR_NPARAMS, s);
        if (loss_out) MP_HIP(hipMemcpyAsync(loss_out, sur->losses.p, sizeof(float), hipMemcpyDeviceToHost, s));
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_surrogate_get_params(mp_surrogate sur, float* params, void* stream) {
    return guarded("mp_surrogate_get_params", [&]() {
        if (!sur || !params) mp_throw(MP_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        copy_out(params, sur->P.p, sizeof(float) * MP_SUR_NPARAMS, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_surrogate_set_params(mp_surrogate sur, const float* params, void* stream) {
    return guarded("mp_surrogate_set_params", [&]() {
        if (!sur || !params) mp_throw(MP_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        std::vector<float> h(MP_SUR_NPARAMS);
        fetch_host(params, sizeof(float) * MP_SUR_NPARAMS, h.data(), s);
        if (!all_finite(h.data(), h.size())) mp_throw(MP_E_ARG, "non-finite weights");
        MP_HIP(hipMemcpyAsync(sur->P.p, h.data(), sizeof(float) * MP_SUR_NPARAMS, hipMemcpyHostToDevice, s));
        mp_sur_reset_adam(sur, s);
        mp_sur_publish(sur, s);
        MP_HIP(hipStreamSynchronize(s));
    });
}

extern "C" mp_status mp_filter_set_surrogate_check(mp_filter f, int32_t period, int32_t stride, float threshold,
                                                   int32_t fallback) {
    return guarded("mp_filter_set_surrogate_check", [&]() {
        if (!f) mp_throw(MP_E_ARG, "null filter");
        if (period < 0 || stride < 1 || fallback < 0 || !(threshold >= 0.0f) || !std::isfinite(threshold))
            mp_throw(MP_E_ARG, "period >= 0, stride >= 1, fallback >= 0 and a finite threshold >= 0 expected");
        if (f->batch_users > 0) mp_throw(MP_E_STATE, "filter held by a batch");
        SurCheck& c = f->chk;
        c.period = period;
        c.stride = stride;
        c.threshold = threshold;
        c.fallback = fallback;
        c.left = 0;
    });
}

extern "C" mp_status mp_filter_set_surrogate(mp_filter f, mp_surrogate sur) {
    return guarded("mp_filter_set_surrogate", [&]() {
        if (!f) mp_throw(MP_E_ARG, "null filter");
        if (sur && sur->map != f->map) mp_throw(MP_E_ARG, "network built for another map");
        if (f->sur) f->sur->users--;
        f->sur = sur;
        if (sur) sur->users++;
    });
}
