// smoother.hip -- smoothing of the representative pose (Sec. IV-A: the
// maximum-posterior particle jitters from frame to frame, which simple
// trajectory smoothing removes).  Host code: no GPU work.
//
// The track holds the last `window` accepted representative poses, each
// carried forward by the motion reported since it was pushed (T <- T dT), so
// that they all estimate the current pose.  A new pose within jump_m /
// jump_rad of the carried newest one is accepted.  A farther one (the
// maximum moved to another mode for a frame, or the filter recovered from a
// kidnap) starts or extends a candidate track; after `switch_frames`
// consecutive far poses that agree with each other the candidate replaces
// the track, otherwise they are held back.  The output is the track's newest
// pose moved by the mean tangent offset of the track:
//   out = T_new exp(mean_i log(T_new^-1 T_i))   (FP64).
#include <array>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>

#include "megapf.h"
#include "mp_internal.hpp"

struct mp_smoother_s {
    mp_smoother_params p{};
    std::deque<std::array<double, 7>> win;    // the track, oldest first
    std::deque<std::array<double, 7>> cand;   // far poses that agree with each other
};

mp_status mp_guarded_call(const char* where, void (*fn)(void*), void* ctx);

namespace {

using Pose = std::array<double, 7>;   // qw qx qy qz tx ty tz

void rot(const double q[4], const double v[3], double o[3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    for (int a = 0; a < 3; ++a) o[a] = R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
}

Pose compose(const Pose& A, const Pose& B) {
    Pose C;
    C[0] = A[0] * B[0] - A[1] * B[1] - A[2] * B[2] - A[3] * B[3];
    C[1] = A[0] * B[1] + A[1] * B[0] + A[2] * B[3] - A[3] * B[2];
    C[2] = A[0] * B[2] - A[1] * B[3] + A[2] * B[0] + A[3] * B[1];
    C[3] = A[0] * B[3] + A[1] * B[2] - A[2] * B[1] + A[3] * B[0];
    double t[3];
    rot(A.data(), B.data() + 4, t);
    for (int a = 0; a < 3; ++a) C[4 + a] = A[4 + a] + t[a];
    const double n = std::sqrt(C[0] * C[0] + C[1] * C[1] + C[2] * C[2] + C[3] * C[3]);
    for (int a = 0; a < 4; ++a) C[a] /= n;
    return C;
}

Pose inverse(const Pose& A) {
    Pose B{A[0], -A[1], -A[2], -A[3], 0, 0, 0};
    double t[3];
    const double mt[3] = {-A[4], -A[5], -A[6]};
    rot(B.data(), mt, t);
    for (int a = 0; a < 3; ++a) B[4 + a] = t[a];
    return B;
}

// SE(3) log / exp with the translation part V(omega)^-1 t / V(omega) v
void se3_log(const Pose& T, double xi[6]) {
    double q[4] = {T[0], T[1], T[2], T[3]};
    if (q[0] < 0)
        for (double& c : q) c = -c;
    const double n = std::sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double th = 2.0 * std::atan2(n, q[0]);
    const double sc = n < 1e-12 ? 2.0 / q[0] : th / n;
    const double w[3] = {sc * q[1], sc * q[2], sc * q[3]};
    const double th2 = th * th;
    const double beta = th2 < 1e-6 ? 1.0 / 12.0 + th2 / 720.0
                                   : (1.0 - 0.5 * th * std::cos(0.5 * th) / std::sin(0.5 * th)) / th2;
    const double* t = T.data() + 4;
    const double c1[3] = {w[1] * t[2] - w[2] * t[1], w[2] * t[0] - w[0] * t[2], w[0] * t[1] - w[1] * t[0]};
    const double c2[3] = {w[1] * c1[2] - w[2] * c1[1], w[2] * c1[0] - w[0] * c1[2], w[0] * c1[1] - w[1] * c1[0]};
    for (int a = 0; a < 3; ++a) {
        xi[a] = w[a];
        xi[3 + a] = t[a] - 0.5 * c1[a] + beta * c2[a];
    }
}

Pose se3_exp(const double xi[6]) {
    const double* w = xi;
    const double* v = xi + 3;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = std::sqrt(th2);
    const double A = th < 1e-5 ? 0.5 - th2 / 24.0 : (1.0 - std::cos(th)) / th2;
    const double B = th < 1e-5 ? 1.0 / 6.0 - th2 / 120.0 : (th - std::sin(th)) / (th2 * th);
    const double hs = th < 1e-5 ? 0.5 - th2 / 48.0 : std::sin(0.5 * th) / th;
    Pose T{th < 1e-5 ? 1.0 - th2 / 8.0 : std::cos(0.5 * th), hs * w[0], hs * w[1], hs * w[2], 0, 0, 0};
    const double c1[3] = {w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2], w[0] * v[1] - w[1] * v[0]};
    const double c2[3] = {w[1] * c1[2] - w[2] * c1[1], w[2] * c1[0] - w[0] * c1[2], w[0] * c1[1] - w[1] * c1[0]};
    for (int a = 0; a < 3; ++a) T[4 + a] = v[a] + A * c1[a] + B * c2[a];
    return T;
}

Pose from_float(const float* p) {
    Pose T;
    for (int a = 0; a < 7; ++a) T[a] = p[a];
    const double n = std::sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2] + T[3] * T[3]);
    for (int a = 0; a < 4; ++a) T[a] /= n;
    return T;
}

bool finite7(const float* p) {
    for (int a = 0; a < 7; ++a)
        if (!std::isfinite(p[a])) return false;
    return (double)p[0] * p[0] + (double)p[1] * p[1] + (double)p[2] * p[2] + (double)p[3] * p[3] > 1e-12;
}

struct CreateCall {
    const mp_smoother_params* p;
    mp_smoother* out;
};
struct PushCall {
    mp_smoother s;
    const float* pose;
    const float* dT;
    float* out;
};

void create_impl(void* ctx) {
    CreateCall& c = *static_cast<CreateCall*>(ctx);
    if (!c.p || !c.out) mp_throw(MP_E_ARG, "null argument");
    if (c.p->window < 1 || c.p->window > 1024 || !(c.p->jump_m > 0.0f) || !(c.p->jump_rad > 0.0f) ||
        c.p->switch_frames < 1 || c.p->switch_frames > 1024)
        mp_throw(MP_E_ARG, "window and switch_frames 1..1024 and positive jump thresholds expected");
    mp_smoother s = new (std::nothrow) mp_smoother_s;
    if (!s) mp_throw(MP_E_OOM, "smoother");
    s->p = *c.p;
    *c.out = s;
}

void push_impl(void* ctx) {
    PushCall& c = *static_cast<PushCall*>(ctx);
    if (!c.s || !c.pose || !c.out) mp_throw(MP_E_ARG, "null argument");
    if (!finite7(c.pose) || (c.dT && !finite7(c.dT))) mp_throw(MP_E_ARG, "non-finite pose or dT, or zero quaternion");
    auto& win = c.s->win;
    auto& cand = c.s->cand;
    if (c.dT) {
        const Pose D = from_float(c.dT);
        for (Pose& T : win) T = compose(T, D);
        for (Pose& T : cand) T = compose(T, D);
    }
    const Pose P = from_float(c.pose);
    auto near = [&](const Pose& A, const Pose& B) {
        const Pose rel = compose(inverse(A), B);
        double d[6];
        se3_log(rel, d);
        const double rot_err = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double tr_err = std::sqrt(rel[4] * rel[4] + rel[5] * rel[5] + rel[6] * rel[6]);
        return tr_err <= c.s->p.jump_m && rot_err <= c.s->p.jump_rad;
    };
    if (win.empty() || near(win.back(), P)) {
        win.push_back(P);
        cand.clear();
    } else {
        if (!cand.empty() && !near(cand.back(), P)) cand.clear();
        cand.push_back(P);
        if ((int)cand.size() >= c.s->p.switch_frames) {   // a persistent new location: switch
            win.swap(cand);
            cand.clear();
        }
    }
    while ((int)win.size() > c.s->p.window) win.pop_front();
    const Pose& Pn = win.back();
    const Pose Pi = inverse(Pn);
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (const Pose& T : win) {
        double d[6];
        se3_log(compose(Pi, T), d);
        for (int a = 0; a < 6; ++a) m[a] += d[a];
    }
    for (double& v : m) v /= (double)win.size();
    const Pose O = compose(Pn, se3_exp(m));
    for (int a = 0; a < 7; ++a) c.out[a] = (float)O[a];
}

void destroy_impl(void* ctx) { delete static_cast<mp_smoother>(ctx); }

}  // namespace

extern "C" void mp_smoother_default_params(mp_smoother_params* p) {
    if (!p) return;
    p->window = 5;
    p->jump_m = 1.0f;
    p->jump_rad = 0.2f;
    p->switch_frames = 3;
}

extern "C" mp_status mp_smoother_create(const mp_smoother_params* p, mp_smoother* out) {
    CreateCall c{p, out};
    return mp_guarded_call("mp_smoother_create", create_impl, &c);
}

extern "C" mp_status mp_smoother_push(mp_smoother s, const float pose[7], const float dT[7], float out[7]) {
    PushCall c{s, pose, dT, out};
    return mp_guarded_call("mp_smoother_push", push_impl, &c);
}

extern "C" mp_status mp_smoother_destroy(mp_smoother s) {
    return mp_guarded_call("mp_smoother_destroy", destroy_impl, s);
}
