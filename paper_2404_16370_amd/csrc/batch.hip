// batch.hip -- several filter instances stepped by one HIP graph replay.
//
// Capture: every instance's step is recorded on its own stream, forked from
// and joined back into the capturing stream, so the graph holds one branch per
// instance.  The kernels of a captured step read the step counter, odometry
// increment and noise factor from a device block (StepDyn per instance) that
// the host refreshes before each replay; every buffer a step touches is sized
// before capture, and the step holds no host synchronisation, allocation or
// memset, so the same graph serves every later step.  Pose buffers ping-pong
// once per SVGD iteration: a captured step with an odd iteration count copies
// the result back to the buffer it started from.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "megapf.h"
#include "mp_internal.hpp"

struct mp_batch_s {
    std::vector<mp_filter> f;
    hipStream_t cap = nullptr;          // capture stream (the caller's may be the null stream)
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr, uploaded = nullptr;
    bool upload_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    StepDyn* host_dyn = nullptr;   // pinned
    DevMem dyn;
    // what each instance looked like when the graph was captured
    struct Shape {
        const void* scan;
        int32_t scan_n, cur;
        const void* partial;
        const void* red;
        const void* hist;
        mp_surrogate sur;
        int32_t lik_batch, lik_layout;
        bool operator!=(const Shape& o) const { return std::memcmp(this, &o, sizeof(Shape)) != 0; }
    };
    std::vector<Shape> shape;
    int32_t captures = 0;
    // persistent likelihood: per iteration one tile queue over the instances
    // whose pass is GROUPED / PLAIN; tables written after each capture
    std::vector<hipEvent_t> pre;        // per instance: its lists are ready
    hipEvent_t lik_done = nullptr;
    DevMem qtab, qfirst, qcount;        // [round][instance] args, [round][instance + 1] first tiles, [round] counters
    int32_t qbatch = 2, qgrid = 0;      // gather batch and workgroups of the queue kernel
    int32_t queued = 0;                 // instances in the queue of the first round
    int64_t queue_tiles = 0;            // tiles per step through the queues
};

namespace {

void release(mp_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipStream_t s : b->branch) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->pre) (void)hipEventDestroy(e);
    if (b->lik_done) (void)hipEventDestroy(b->lik_done);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->host_dyn) (void)hipHostFree(b->host_dyn);
    for (mp_filter f : b->f) f->batch_users--;
    delete b;
}

mp_batch_s::Shape shape_of(mp_filter f) {
    mp_batch_s::Shape s;
    std::memset(&s, 0, sizeof(s));
    s.scan = f->scan.p;
    s.scan_n = f->scan_n;
    s.cur = f->cur;
    s.partial = f->partial.p;
    s.red = f->red.p;
    s.hist = f->hist.p;
    s.sur = f->sur;
    s.lik_batch = f->p.lik_batch;
    s.lik_layout = f->p.lik_layout;
    return s;
}

void check_ready(mp_filter f) {
    if (f->scan_n < 0) mp_throw(MP_E_STATE, "every instance needs a scan (mp_scan_upload)");
    if (f->p.scorer == MP_SCORER_SURROGATE && !f->sur)
        mp_throw(MP_E_STATE, "SURROGATE scorer without a network (mp_filter_set_surrogate)");
    if (f->p.scorer == MP_SCORER_SURROGATE && f->chk.period > 0)
        mp_throw(MP_E_UNSUPPORTED, "the surrogate check reads its verdict on the host: not in a batch");
}

void capture(mp_batch b, hipStream_t caller) {
    for (mp_filter f : b->f) mp_reserve_step(f);
    // buffers just sized may still be in use by queued work of the caller
    MP_HIP(hipStreamSynchronize(caller));
    hipStream_t s = b->cap;
    if (b->exec) {
        MP_HIP(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    if (b->graph) {
        MP_HIP(hipGraphDestroy(b->graph));
        b->graph = nullptr;
    }
    b->shape.clear();
    const size_t n = b->f.size();
    int rounds = 0;
    for (mp_filter f : b->f)
        if (f->scan_n > 0) rounds = std::max(rounds, f->p.svgd_iters);
    const size_t argb = mp_lik_args_bytes();
    b->qtab.ensure(std::max<size_t>(1, (size_t)rounds * n) * argb);
    b->qfirst.ensure(sizeof(int32_t) * std::max<size_t>(1, (size_t)rounds * (n + 1)));
    b->qcount.ensure(sizeof(int32_t) * std::max(1, rounds));
    if (b->qgrid <= 0) b->qgrid = mp_lik_queue_grid(b->qbatch);
    std::vector<char> htab((size_t)rounds * n * argb);
    std::vector<int32_t> hfirst((size_t)rounds * (n + 1), 0);
    std::vector<int> start(n);
    for (size_t i = 0; i < n; ++i) start[i] = b->f[i]->cur;
    b->queued = 0;
    b->queue_tiles = 0;
    MP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        MP_HIP(hipEventRecord(b->fork, s));
        for (size_t i = 0; i < n; ++i) {
            mp_filter f = b->f[i];
            MP_HIP(hipStreamWaitEvent(b->branch[i], b->fork, 0));
            start[i] = f->cur;
            b->shape.push_back(shape_of(f));
            f->capturing = true;
            f->dyn = b->dyn.as<StepDyn>() + i;
            mp_step_begin(f, false, nullptr, nullptr, false, b->branch[i]);
        }
        // the correction iterations in lock step: every instance's lists, then
        // one persistent launch over the tiles of all queued likelihood passes,
        // then each instance's solve and SVGD update
        for (int it = 0; it < rounds; ++it) {
            std::vector<size_t> queued;
            int32_t tiles = 0;
            for (size_t i = 0; i < n; ++i) {
                mp_filter f = b->f[i];
                if (f->scan_n <= 0 || it >= f->p.svgd_iters) continue;
                hipStream_t bs = b->branch[i];
                mp_step_iter_nbr(f, it, bs);
                int32_t t = 0;
                char* slot = htab.data() + ((size_t)it * n + queued.size()) * argb;
                if (mp_lik_queue_plan(f, slot, &t, bs)) {
                    hfirst[(size_t)it * (n + 1) + queued.size()] = tiles;
                    tiles += t;
                    queued.push_back(i);
                    MP_HIP(hipEventRecord(b->pre[i], bs));
                    MP_HIP(hipStreamWaitEvent(s, b->pre[i], 0));
                } else {
                    mp_launch_likelihood(f, bs);
                }
            }
            if (!queued.empty()) {
                int32_t* counter = b->qcount.as<int32_t>() + it;
                mp_fill_u32(counter, 0u, 1, s);
                mp_launch_lik_queue(b->qtab.as<char>() + (size_t)it * n * argb,
                                    b->qfirst.as<int32_t>() + (size_t)it * (n + 1), counter, (int)queued.size(),
                                    tiles, b->qbatch, b->qgrid, s);
                MP_HIP(hipEventRecord(b->lik_done, s));
                for (size_t i : queued) {
                    MP_HIP(hipStreamWaitEvent(b->branch[i], b->lik_done, 0));
                    mp_lik_queue_solve(b->f[i], b->branch[i]);
                }
                if (it == 0) b->queued = (int32_t)queued.size();
                b->queue_tiles += tiles;
            }
            for (size_t i = 0; i < n; ++i) {
                mp_filter f = b->f[i];
                if (f->scan_n <= 0 || it >= f->p.svgd_iters) continue;
                mp_step_iter_svgd(f, it, b->branch[i]);
            }
        }
        for (size_t i = 0; i < n; ++i) {
            mp_filter f = b->f[i];
            hipStream_t bs = b->branch[i];
            mp_step_end(f, bs);
            if (f->cur != start[i]) {
                mp_copy_poses(f, f->cur, start[i], bs);
                f->cur = start[i];
            }
            f->capturing = false;
            f->dyn = nullptr;
            MP_HIP(hipEventRecord(b->join[i], bs));
            MP_HIP(hipStreamWaitEvent(s, b->join[i], 0));
        }
    } catch (...) {
        for (size_t i = 0; i < n; ++i) {
            b->f[i]->capturing = false;
            b->f[i]->dyn = nullptr;
            b->f[i]->cur = start[i];
        }
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        b->shape.clear();
        throw;
    }
    MP_HIP(hipStreamEndCapture(s, &b->graph));
    MP_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    // the queue tables hold pointers and sizes that stay fixed while the graph does
    if (rounds > 0) {
        MP_HIP(hipMemcpyAsync(b->qtab.p, htab.data(), htab.size(), hipMemcpyHostToDevice, caller));
        MP_HIP(hipMemcpyAsync(b->qfirst.p, hfirst.data(), sizeof(int32_t) * hfirst.size(), hipMemcpyHostToDevice,
                              caller));
        MP_HIP(hipStreamSynchronize(caller));
    }
    b->captures++;
}

// time the likelihood launch of each (layout, gather batch) candidate and keep
// the fastest; both choices change speed only (same per-point arithmetic)
void autotune(mp_filter f, hipStream_t s) {
    if (f->scan_n <= 0 || f->p.scorer != MP_SCORER_PLAIN) return;
    hipEvent_t e0, e1;
    MP_HIP(hipEventCreate(&e0));
    MP_HIP(hipEventCreate(&e1));
    const int32_t keep_b = f->p.lik_batch, keep_l = f->p.lik_layout;
    int32_t best_b = keep_b, best_l = keep_l;
    float best_ms = 1e30f;
    static const int32_t cand[][2] = {{MP_LIK_LAYOUT_PARTICLE, 2}, {MP_LIK_LAYOUT_PARTICLE, 4},
                                      {MP_LIK_LAYOUT_PARTICLE, 8}, {MP_LIK_LAYOUT_PARTICLE, 16},
                                      {MP_LIK_LAYOUT_GROUPED, 2},  {MP_LIK_LAYOUT_GROUPED, 4},
                                      {MP_LIK_LAYOUT_GROUPED, 8}};
    try {
        for (const auto& c : cand) {
            f->p.lik_layout = c[0];
            f->p.lik_batch = c[1];
            mp_launch_likelihood(f, s);   // warm-up (sizes the partial buffer)
            MP_HIP(hipEventRecord(e0, s));
            mp_launch_likelihood(f, s);
            mp_launch_likelihood(f, s);
            MP_HIP(hipEventRecord(e1, s));
            MP_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            MP_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best_l = c[0];
                best_b = c[1];
            }
        }
    } catch (...) {
        f->p.lik_batch = keep_b;
        f->p.lik_layout = keep_l;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    f->p.lik_batch = best_b;
    f->p.lik_layout = best_l;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

bool queue_eligible(mp_filter f) {
    return f->p.scorer == MP_SCORER_PLAIN && f->map->view.backend == MP_NNF_DENSE;
}

// time the persistent likelihood over the instances' current passes for each
// gather batch and keep the fastest (speed only: a lane's points and their
// order are the same for every batch)
void tune_queue(mp_batch b, hipStream_t s) {
    const size_t n = b->f.size(), argb = mp_lik_args_bytes();
    std::vector<char> tab(n * argb);
    std::vector<int32_t> first(n + 1, 0);
    int32_t tiles = 0, q = 0;
    for (mp_filter f : b->f) {
        int32_t t = 0;
        if (mp_lik_queue_plan(f, tab.data() + (size_t)q * argb, &t, s)) {
            first[q++] = tiles;
            tiles += t;
        }
    }
    if (q == 0) return;
    DevMem dtab, dfirst, dcnt;
    dtab.alloc(tab.size());
    dfirst.alloc(sizeof(int32_t) * first.size());
    dcnt.alloc(sizeof(int32_t));
    MP_HIP(hipMemcpyAsync(dtab.p, tab.data(), tab.size(), hipMemcpyHostToDevice, s));
    MP_HIP(hipMemcpyAsync(dfirst.p, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    MP_HIP(hipEventCreate(&e0));
    MP_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    try {
        for (int batch : {2, 4, 8}) {
            const int grid = mp_lik_queue_grid(batch);
            for (int rep = 0; rep < 3; ++rep) {   // the first is a warm-up
                if (rep == 1) MP_HIP(hipEventRecord(e0, s));
                mp_fill_u32(dcnt.p, 0u, 1, s);
                mp_launch_lik_queue(dtab.p, dfirst.as<int32_t>(), dcnt.as<int32_t>(), q, tiles, batch, grid, s);
            }
            MP_HIP(hipEventRecord(e1, s));
            MP_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            MP_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                b->qbatch = batch;
                b->qgrid = grid;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

mp_status mp_guarded_call(const char* where, void (*fn)(void*), void* ctx);

namespace {
struct CreateCtx {
    const mp_filter* filters;
    int32_t n, tune;
    hipStream_t s;
    mp_batch* out;
};
void create_impl(void* p) {
    CreateCtx& c = *static_cast<CreateCtx*>(p);
    if (!c.filters || !c.out || c.n < 1) mp_throw(MP_E_ARG, "need at least one filter");
    for (int32_t i = 0; i < c.n; ++i) {
        if (!c.filters[i]) mp_throw(MP_E_ARG, "null filter");
        check_ready(c.filters[i]);
        for (int32_t j = 0; j < i; ++j)
            if (c.filters[j] == c.filters[i]) mp_throw(MP_E_STATE, "a filter appears twice in the batch");
    }
    mp_batch b = new mp_batch_s();
    try {
        for (int32_t i = 0; i < c.n; ++i) {
            b->f.push_back(c.filters[i]);
            c.filters[i]->batch_users++;
            hipStream_t st;
            MP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            b->branch.push_back(st);
            hipEvent_t e;
            MP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->join.push_back(e);
            MP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->pre.push_back(e);
        }
        MP_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        MP_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        MP_HIP(hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming));
        MP_HIP(hipEventCreateWithFlags(&b->lik_done, hipEventDisableTiming));
        MP_HIP(hipHostMalloc(reinterpret_cast<void**>(&b->host_dyn), sizeof(StepDyn) * (size_t)c.n,
                             hipHostMallocDefault));
        b->dyn.alloc(sizeof(StepDyn) * (size_t)c.n);
        // PLAIN instances on dense maps take the GROUPED layout, so that their
        // likelihood passes join the persistent tile queue; the others keep
        // their own launches (autotuned per instance)
        for (mp_filter f : b->f)
            if (queue_eligible(f)) f->p.lik_layout = MP_LIK_LAYOUT_GROUPED;
        if (c.tune) {
            for (mp_filter f : b->f)
                if (!queue_eligible(f)) autotune(f, c.s);
            tune_queue(b, c.s);
        }
        MP_HIP(hipStreamSynchronize(c.s));
    } catch (...) {
        release(b);
        throw;
    }
    *c.out = b;
}

struct StepCtx {
    mp_batch b;
    const float* dT;
    const float* cov;
    hipStream_t s;
};
void step_impl(void* p) {
    StepCtx& c = *static_cast<StepCtx*>(p);
    mp_batch b = c.b;
    if (!b) mp_throw(MP_E_ARG, "null batch");
    const size_t n = b->f.size();
    for (mp_filter f : b->f) check_ready(f);
    // step values of every instance (validated before anything is launched)
    std::vector<StepDyn> d(n);
    for (size_t i = 0; i < n; ++i) {
        mp_filter f = b->f[i];
        std::memset(&d[i], 0, sizeof(StepDyn));
        d[i].frame = (uint32_t)f->frame;
        d[i].dq[0] = 1.0f;
        if (c.dT) {
            float dq[7], L[36];
            bool noise = false;
            mp_prepare_prediction(c.dT + 7 * i, c.cov ? c.cov + 36 * i : nullptr, dq, L, noise);
            d[i].do_pred = 1;
            d[i].noise = noise ? 1 : 0;
            for (int k = 0; k < 4; ++k) d[i].dq[k] = dq[k];
            for (int k = 0; k < 3; ++k) d[i].dt[k] = dq[4 + k];
            int q = 0;
            for (int r = 0; r < 6; ++r)
                for (int cc = 0; cc <= r; ++cc) d[i].L[q++] = noise ? L[6 * r + cc] : 0.0f;
        }
    }
    bool recapture = !b->exec || b->shape.size() != n;
    for (size_t i = 0; i < n && !recapture; ++i) {
        mp_reserve_step(b->f[i]);
        recapture = shape_of(b->f[i]) != b->shape[i];
    }
    if (recapture) capture(b, c.s);
    // the pinned block may still be read by the previous call's copy
    if (b->upload_pending) MP_HIP(hipEventSynchronize(b->uploaded));
    std::memcpy(b->host_dyn, d.data(), sizeof(StepDyn) * n);
    MP_HIP(hipMemcpyAsync(b->dyn.p, b->host_dyn, sizeof(StepDyn) * n, hipMemcpyHostToDevice, c.s));
    MP_HIP(hipEventRecord(b->uploaded, c.s));
    b->upload_pending = true;
    MP_HIP(hipGraphLaunch(b->exec, c.s));
    for (size_t i = 0; i < n; ++i) {
        mp_filter f = b->f[i];
        for (int st = 0; st < MP_NUM_STAGES; ++st)
            if (st != MP_STAGE_SCAN) f->ev_count[st] = 0;
        f->frame++;
        f->last_stream = c.s;
    }
}
}  // namespace

extern "C" mp_status mp_batch_create(const mp_filter* filters, int32_t n, int32_t tune, void* stream,
                                     mp_batch* out) {
    CreateCtx c{filters, n, tune, static_cast<hipStream_t>(stream), out};
    return mp_guarded_call("mp_batch_create", create_impl, &c);
}

extern "C" mp_status mp_batch_step(mp_batch b, const float* dT, const float* cov_dT, void* stream) {
    StepCtx c{b, dT, cov_dT, static_cast<hipStream_t>(stream)};
    return mp_guarded_call("mp_batch_step", step_impl, &c);
}

namespace {
struct InfoCtx {
    mp_batch b;
    mp_batch_info* out;
    int32_t* lb;
    int32_t* ll;
};
void info_impl(void* p) {
    InfoCtx& c = *static_cast<InfoCtx*>(p);
    if (!c.b || !c.out) mp_throw(MP_E_ARG, "null argument");
    c.out->n_instances = (int32_t)c.b->f.size();
    c.out->captures = c.b->captures;
    int64_t ev = 0;
    for (size_t i = 0; i < c.b->f.size(); ++i) {
        mp_filter f = c.b->f[i];
        const int passes = f->p.svgd_iters + (f->p.svgd_iters > 0 && f->p.final_rescore ? 1 : 0);
        ev += (int64_t)f->n * std::max(0, f->scan_n) * passes;
        if (c.lb) c.lb[i] = f->p.lik_batch;
        if (c.ll) c.ll[i] = f->p.lik_layout;
    }
    c.out->evals_per_step = ev;
    c.out->queued_instances = c.b->queued;
    c.out->queue_batch = c.b->qbatch;
    c.out->queue_workgroups = c.b->qgrid;
    c.out->queue_tiles_per_step = c.b->queue_tiles;
}
void destroy_impl(void* p) {
    mp_batch b = static_cast<mp_batch>(p);
    if (!b) return;
    MP_HIP(hipDeviceSynchronize());
    release(b);
}
}  // namespace

extern "C" mp_status mp_batch_get_info(mp_batch b, mp_batch_info* out, int32_t* lik_batch_out,
                                       int32_t* lik_layout_out) {
    InfoCtx c{b, out, lik_batch_out, lik_layout_out};
    return mp_guarded_call("mp_batch_get_info", info_impl, &c);
}

extern "C" mp_status mp_batch_destroy(mp_batch b) { return mp_guarded_call("mp_batch_destroy", destroy_impl, b); }
