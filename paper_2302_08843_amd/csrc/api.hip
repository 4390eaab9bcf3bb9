// api.hip -- the C ABI declared in include/mm.h: plan life cycle, argument
// checks, and the host-side step-size controller of the Dormand-Prince
// integrator (the device computes the stages, the error norm and the torque;
// the host receives 8 bytes per step and decides).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "engine.h"

namespace mmx {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int padded_extent(int n)
{
    if (n <= 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return p;
}

static size_t elem_size(const Plan& p) { return p.prec == MM_FP32 ? 4 : 8; }

mm_status hip_fail(hipError_t e, const char* what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EHIP;
}

#define MM_HIP(call, what)                               \
    do {                                                 \
        hipError_t e__ = (call);                         \
        if (e__ != hipSuccess) return hip_fail(e__, what); \
    } while (0)

void free_plan(Plan* p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    if (p->ws) {
        // carved from the caller's workspace: not ours to free
        p->Khat = p->S1 = p->S2 = p->tw = p->rk = nullptr;
        p->red = p->red_out = nullptr;
        p->ctl = nullptr;
        p->epart = nullptr;
    }
    for (auto& r : p->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : p->prof.pool) (void)hipEventDestroy(e);
    if (p->shared) {
        release_tensor(p->shared);
        p->Khat = p->tw = nullptr;
    }
    if (p->st64) (void)hipFree(p->st64);
    if (p->Pb) (void)hipFree(p->Pb);
    if (p->Ms_b) (void)hipFree(p->Ms_b);
    if (p->Pb_host) (void)hipHostFree(p->Pb_host);
    void* bufs[] = {p->Khat, p->S1, p->S2 == p->S1 ? nullptr : p->S2, p->tw, p->Ms_cell,
                    p->A_cell, p->D_cell, p->Ku_cell, p->zw, p->lw, p->oe_G, p->h_oe, p->mask, p->rk, p->red, p->red_out, p->adj, p->seg,
                    p->gms, p->ctl, p->epart};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->host_out) (void)hipHostFree(p->host_out);
    delete p;
}

void release_tensor(SharedTensor* t)
{
    if (!t || --t->refs > 0) return;
    if (t->Khat) (void)hipFree(t->Khat);
    if (t->tw) (void)hipFree(t->tw);
    delete t;
}

static mm_status alloc(Plan* p, void** out, size_t bytes, const char* what)
{
    hipError_t e = hipMalloc(out, bytes ? bytes : 1);
    if (e != hipSuccess) return hip_fail(e, what);
    p->bytes += bytes;
    return MM_OK;
}

// Dormand & Prince (1980) 5(4) coefficients.
static const double kC[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double kA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
static const double kB5[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                              -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double kB4[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                              -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

// Runge-Kutta-Fehlberg 4(5) (Fehlberg 1969): 4th-order solution propagated.
static const double kFC[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double kFA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0}};
static const double kFB4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double kFB5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                               -9.0 / 50.0, 2.0 / 55.0};

// An embedded pair as the controller uses it: stage count, nodes, rows of
// coefficients, propagated weights b, error weights e; fsal: the last stage's
// input is the propagated solution and its derivative the next first stage.
struct Tableau {
    int stages;
    bool fsal;
    const double* c;
    const double* a[7];
    double b[7], e[7];
};

static Tableau tableau(int method)
{
    Tableau T{};
    if (method == MM_RKF45) {
        T.stages = 6;
        T.fsal = false;
        T.c = kFC;
        for (int s = 0; s < 6; ++s) {
            T.a[s] = kFA[s];
            T.b[s] = kFB4[s];
            T.e[s] = kFB4[s] - kFB5[s];
        }
    } else {
        T.stages = 7;
        T.fsal = true;
        T.c = kC;
        for (int s = 0; s < 7; ++s) {
            T.a[s] = kA[s];
            T.b[s] = kB5[s];
            T.e[s] = kB5[s] - kB4[s];
        }
    }
    return T;
}

mm_status ensure_rk(Plan* p)
{
    // a batch plan holds every request's vectors and controller
    const size_t nb = (size_t)p->batch;
    if (!p->rk) {
        mm_status s = alloc(p, &p->rk, 10 * 3 * (size_t)p->N * nb * elem_size(*p),
                            "Runge-Kutta buffers");
        if (s != MM_OK) return s;
    }
    if (p->state64 && !p->st64) {
        mm_status s = alloc(p, (void**)&p->st64, 6 * sizeof(double) * (size_t)p->N * nb,
                            "double state");
        if (s != MM_OK) return s;
    }
    if (!p->ctl) return alloc(p, (void**)&p->ctl, sizeof(DevCtl) * nb, "step controller");
    return MM_OK;
}

// Error-norm partials of the last stage's local pass (one pair per block, at
// most one block per x row), for host-controlled steps (part of a caller
// workspace, else allocated on first use).
static bool ensure_epart(Plan* p)
{
    if (p->epart) return true;
    if (p->ws || p->Pb) return false;
    return alloc(p, (void**)&p->epart, 2 * sizeof(double) * (size_t)p->n[1] * p->n[2],
                 "error-norm partials") == MM_OK;
}

// Elements between consecutive Runge-Kutta vectors (and between y and y1 of
// the double state): 3N, or the whole batch's 3N per vector.
static long vec_stride(const Plan* p) { return p->vstride ? p->vstride : 3 * p->N; }

template <typename T>
static T* rk_vec(Plan* p, int i)
{
    return (T*)p->rk + (size_t)i * vec_stride(p);
}

// The stage input y + h sum_{j < nk} a_j k_j written to ys (h read from hdev
// on the device when hdev is not null), coefficients as rk_combine forms them.
template <typename T>
static StageIn<T> stage_in(const T* y, T* const* k, const double* a, int nk, double h,
                           const double* hdev, T* ys)
{
    StageIn<T> sc;
    sc.y = y;
    sc.ys = ys;
    sc.nk = nk;
    sc.h = hdev;
    for (int j = 0; j < nk; ++j) {
        sc.k[j] = k[j];
        sc.c[j] = hdev ? a[j] : h * a[j];
    }
    return sc;
}

static mm_status fetch(Plan* p, int n)
{
    MM_HIP(hipMemcpyAsync(p->host_out, p->red_out, sizeof(double) * n, hipMemcpyDeviceToHost,
                          p->stream),
           "reading a reduction");
    MM_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
    return MM_OK;
}

static mm_status ensure_adj(Plan* p)
{
    if (!p->adj) {
        mm_status s = alloc(p, &p->adj, 16 * 3 * (size_t)p->N * elem_size(*p), "adjoint buffers");
        if (s != MM_OK) return s;
    }
    if (!p->gms) {
        mm_status s = alloc(p, (void**)&p->gms, sizeof(double) * (size_t)p->N, "Ms gradient");
        if (s != MM_OK) return s;
    }
    return MM_OK;
}

template <typename T>
static T* adj_vec(Plan* p, int i)
{
    return (T*)p->adj + (size_t)i * 3 * p->N;
}

// Hairer-Norsett-Wanner starting step from y and f0 = f(t, y) (one extra
// right-hand side into f1, using ys as scratch).  Synchronises twice.
template <typename T>
static mm_status start_step(Plan* p, const T* y, T* f0, T* f1, T* ys, const double hext[3],
                            unsigned terms, double t, double alpha, bool precess, double rtol,
                            double atol, double* dt, long* evals)
{
    MM_HIP(start_norms<T>(*p, y, f0, nullptr, rtol, atol, p->red_out + 2), "start norms");
    mm_status s = fetch(p, 5);
    if (s != MM_OK) return s;
    const double cnt = 3.0 * (double)p->n_magnetic;
    const double d0 = cnt > 0 ? std::sqrt(p->host_out[2] / cnt) : 0.0;
    const double d1 = cnt > 0 ? std::sqrt(p->host_out[3] / cnt) : 0.0;
    const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    const double one = 1.0;
    T* fs = f0;
    MM_HIP(rk_combine<T>(*p, ys, y, h0, &one, &fs, 1), "start step");
    MM_HIP(eval_field<T>(*p, ys, hext, terms, t + h0, nullptr, f1, alpha, precess, nullptr),
           "right-hand side");
    (*evals)++;
    MM_HIP(start_norms<T>(*p, y, f0, f1, rtol, atol, p->red_out + 2), "start norms");
    s = fetch(p, 5);
    if (s != MM_OK) return s;
    const double d2 = (cnt > 0 ? std::sqrt(p->host_out[4] / cnt) : 0.0) / h0;
    const double mx = std::max(d1, d2);
    const double h1 = mx <= 1e-15 ? std::max(1e-6, h0 * 1e-3) : std::pow(0.01 / mx, 0.2);
    *dt = std::min(100.0 * h0, h1);
    return MM_OK;
}

// ---------------------------------------------------------------------------
// Device-controlled Dormand-Prince steps (used by the request server): the
// state stays in rk vector 8, the trial state in 9, stage derivatives in 0..6
// and the stage input in 7; the controller state is p->ctl.  With a double
// state (Plan::state64) the state and trial state live in p->st64, vector 7
// holds the float stage input, which between steps is the rounded state, and
// vector 8 its rounding residual.
// ---------------------------------------------------------------------------
template <typename T>
mm_status dev_prepare(Plan* p, const void* m0, const double hext[3], unsigned terms,
                      const DevCtl& init, double rtol, double atol)
{
    mm_status s = ensure_rk(p);
    if (s != MM_OK) return s;
    const bool relax = init.relax != 0;
    const double alpha = relax ? 1.0 : p->alpha;
    const bool d64 = std::is_same<T, float>::value && p->state64;
    // the state the fields are evaluated at: vector 8, or with a double
    // state its float copy in vector 7
    T* y = rk_vec<T>(p, d64 ? 7 : 8);
    T* k0 = rk_vec<T>(p, 0);
    MM_HIP(hipMemcpyAsync(y, m0, 3 * (size_t)p->N * sizeof(T), hipMemcpyDeviceToDevice, p->stream),
           "copy m");
    if (d64) MM_HIP(convert_f32_f64(*p, (const float*)y, p->st64, 3 * p->N), "double state");
    MM_HIP(eval_field<T>(*p, y, hext, terms, init.t, nullptr, k0, alpha, !relax,
                         relax ? p->red_out + 1 : nullptr),
           "right-hand side");
    DevCtl c = init;
    c.rhs_evals = 1;
    if (!(c.dt > 0.0)) {
        s = start_step<T>(p, y, k0, rk_vec<T>(p, 1), rk_vec<T>(p, d64 ? 9 : 7), hext, terms, c.t,
                          alpha, !relax, rtol, atol, &c.dt, &c.rhs_evals);
        if (s != MM_OK) return s;
    }
    c.torque = std::numeric_limits<double>::infinity();
    MM_HIP(hipMemcpyAsync(p->ctl, &c, sizeof(DevCtl), hipMemcpyHostToDevice, p->stream), "controller");
    if (relax) MM_HIP(dp_torque(*p, p->ctl), "torque");
    // the controller copy reads from the stack: finish it before returning
    MM_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
    return MM_OK;
}

// One device-controlled step (no host synchronisation; capturable).  Fields
// must not depend on time (no drive).
template <typename T>
mm_status dev_step(Plan* p, const double hext[3], unsigned terms, double rtol, double atol,
                   bool relax, bool renorm)
{
    const double alpha = relax ? 1.0 : p->alpha;
    T* k[7];
    for (int i = 0; i < 7; ++i) k[i] = rk_vec<T>(p, i);
    T* ys = rk_vec<T>(p, 7);
    T* y = rk_vec<T>(p, 8);
    T* y1 = rk_vec<T>(p, 9);
    double* hdev = &p->ctl->h;
    MM_HIP(dp_begin(*p, p->ctl), "controller");
    if constexpr (std::is_same<T, float>::value) {
        if (p->state64) {
            // double state: stage inputs formed in double and evaluated in
            // float, the rounding residual (vector 8, free with a double
            // state) carried into the exchange differences
            double* yd = p->st64;
            double* y1d = p->st64 + vec_stride(p);
            T* ys_lo = y;
            for (int sg = 1; sg < 7; ++sg) {
                MM_HIP(rk_combine_d(*p, ys, sg == 6 ? y1d : nullptr, yd, kA[sg], k, sg, hdev,
                                    ys_lo),
                       "stage input");
                MM_HIP(eval_field<T>(*p, ys, hext, terms, 0.0, nullptr, k[sg], alpha, !relax,
                                     nullptr, ys_lo),
                       "right-hand side");
            }
            double E[7];
            for (int j = 0; j < 7; ++j) E[j] = kB5[j] - kB4[j];
            MM_HIP(rk_error_norm_d(*p, yd, y1d, E, k, 7, rtol, atol, p->red_out, hdev, p->ctl),
                   "error norm and controller");
            MM_HIP(dp_commit_d(*p, p->ctl, yd, y1d, ys, k[0], k[6], ys_lo), "commit");
            // the closing evaluation leaves the torque for the next step's
            // begin
            if (renorm)
                MM_HIP(eval_field<T>(*p, ys, hext, terms, 0.0, nullptr, k[0], alpha, !relax,
                                     relax ? p->red_out + 1 : nullptr, ys_lo),
                       "right-hand side");
            return MM_OK;
        }
    }
    for (int sg = 1; sg < 7; ++sg) {
        const StageIn<T> sc = stage_in<T>(y, k, kA[sg], sg, 0.0, hdev, sg == 6 ? y1 : ys);
        MM_HIP(eval_field_stage<T>(*p, sc, hext, terms, 0.0, k[sg], alpha, !relax, nullptr),
               "right-hand side");
    }
    double E[7];
    for (int j = 0; j < 7; ++j) E[j] = kB5[j] - kB4[j];
    MM_HIP(rk_error_norm<T>(*p, y, y1, 0.0, E, k, 7, rtol, atol, p->red_out, hdev, p->ctl),
           "error norm and controller");
    MM_HIP(dp_commit<T>(*p, p->ctl, y, y1, k[0], k[6]), "commit");
    // the closing evaluation leaves the torque for the next step's begin
    if (renorm)
        MM_HIP(eval_field<T>(*p, y, hext, terms, 0.0, nullptr, k[0], alpha, !relax,
                             relax ? p->red_out + 1 : nullptr),
               "right-hand side");
    return MM_OK;
}

template <typename T>
T* dev_state(Plan* p)
{
    return rk_vec<T>(p, 8);
}

hipError_t dev_result(Plan* p, void* out)
{
    if (p->prec == MM_FP32 && p->state64)
        return convert_f64_f32(*p, p->st64, (float*)out, 3 * p->N);
    const size_t vb = 3 * (size_t)p->N * elem_size(*p);
    const void* y = p->prec == MM_FP32 ? (const void*)rk_vec<float>(p, 8)
                                       : (const void*)rk_vec<double>(p, 8);
    return hipMemcpyAsync(out, y, vb, hipMemcpyDeviceToDevice, p->stream);
}

size_t state64_bytes(const int grid[3])
{
    return 6 * sizeof(double) * (size_t)grid[0] * grid[1] * grid[2];
}

template mm_status dev_prepare<float>(Plan*, const void*, const double*, unsigned, const DevCtl&,
                                      double, double);
template mm_status dev_prepare<double>(Plan*, const void*, const double*, unsigned, const DevCtl&,
                                       double, double);
template mm_status dev_step<float>(Plan*, const double*, unsigned, double, double, bool, bool);
template mm_status dev_step<double>(Plan*, const double*, unsigned, double, double, bool, bool);
template float* dev_state<float>(Plan*);
template double* dev_state<double>(Plan*);

// ---------------------------------------------------------------------------
// Dormand-Prince integrator loop.  mode_relax: alpha = 1, no precession, renormalise,
// stop on the torque criterion.
// ---------------------------------------------------------------------------
template <typename T>
static mm_status dp45(Plan* p, void* m_user, const double hext[3], unsigned terms, double* t,
                      double* dt, double rtol, double atol, double t_end, long max_steps,
                      double dt_min, bool renorm, bool relax, double torque_tol,
                      mm_step_stats* st, int method = MM_DP45)
{
    const Tableau TB = tableau(method);
    const int S = TB.stages;
    mm_status s = ensure_rk(p);
    if (s != MM_OK) return s;
    const double alpha = relax ? 1.0 : p->alpha;
    const bool precess = !relax;
    T* k[7];
    for (int i = 0; i < 7; ++i) k[i] = rk_vec<T>(p, i);
    T* ys = rk_vec<T>(p, 7);
    T* y = rk_vec<T>(p, 8);
    T* y1 = rk_vec<T>(p, 9);
    const size_t vbytes = 3 * (size_t)p->N * sizeof(T);
    mm_step_stats loc{};
    mm_status status = MM_OK;
    double* torque_dev = relax ? p->red_out + 1 : nullptr;

    MM_HIP(hipMemcpyAsync(y, m_user, vbytes, hipMemcpyDeviceToDevice, p->stream), "copy m");
    MM_HIP(eval_field<T>(*p, y, hext, terms, *t, nullptr, k[0], alpha, precess, torque_dev),
           "right-hand side");
    loc.rhs_evals++;
    if (*dt <= 0.0) {
        s = start_step<T>(p, y, k[0], k[1], ys, hext, terms, *t, alpha, precess, rtol, atol, dt,
                          &loc.rhs_evals);
        if (s != MM_OK) return s;
    }
    bool last_rejected = false;
    double torque = std::numeric_limits<double>::infinity();
    bool torque_known = false;
    // Dormand-Prince (first-same-as-last, 7 stages): the error norm is
    // accumulated by the last stage's passes where the plan allows it
    const bool fuse_err = TB.fsal && S == 7 && ensure_epart(p) && err_fusable(*p, terms);
    while (loc.accepted < max_steps && *t < t_end) {
        if (relax) {
            if (!torque_known) {
                s = fetch(p, 2);
                if (s != MM_OK) break;
                torque = p->host_out[1];
                torque_known = true;
            }
            if (torque < torque_tol) break;
        }
        double h = *dt;
        if (*t + h > t_end) h = t_end - *t;
        for (int sg = 1; sg < S; ++sg) {
            T* target = (TB.fsal && sg == S - 1) ? y1 : ys;
            StageIn<T> sc = stage_in<T>(y, k, TB.a[sg], sg, h, nullptr, target);
            if (fuse_err && sg == S - 1) {
                // the last stage's x forward pass also forms the partial error
                // of the first six derivatives (into the free stage-input
                // vector) and its local pass adds the seventh and reduces
                sc.ep = ys;
                for (int j = 0; j < sg; ++j) sc.e[j] = h * TB.e[j];
                ErrIn<T> ei;
                ei.y = y;
                ei.e6 = h * TB.e[sg];
                ei.rtol = rtol;
                ei.atol = atol;
                ei.out_dev = p->red_out;
                MM_HIP(eval_field_stage<T>(*p, sc, hext, terms, *t + TB.c[sg] * h, k[sg], alpha,
                                           precess, nullptr, &ei),
                       "right-hand side and error norm");
            } else {
                MM_HIP(eval_field_stage<T>(*p, sc, hext, terms, *t + TB.c[sg] * h, k[sg], alpha,
                                           precess, nullptr),
                       "right-hand side");
            }
            loc.rhs_evals++;
        }
        if (!TB.fsal) MM_HIP(rk_combine<T>(*p, y1, y, h, TB.b, k, S), "solution");
        if (!fuse_err)
            MM_HIP(rk_error_norm<T>(*p, y, y1, h, TB.e, k, S, rtol, atol, p->red_out),
                   "error norm");
        s = fetch(p, 6);
        if (s != MM_OK) break;
        double err = p->host_out[0];
        loc.err_last = err;
        if (!std::isfinite(err)) {
            // an overflowing trial step is rejected with the minimum factor;
            // only a non-finite current state is an error
            if (p->host_out[5] != 0.0) {
                set_error("non-finite magnetisation");
                status = MM_ENONFINITE;
                break;
            }
            err = std::numeric_limits<double>::infinity();
        }
        if (err <= 1.0) {
            *t += h;
            std::swap(y, y1);
            loc.accepted++;
            if (renorm || !TB.fsal) {
                if (renorm) MM_HIP(renormalise<T>(*p, y), "renormalise");
                MM_HIP(eval_field<T>(*p, y, hext, terms, *t, nullptr, k[0], alpha, precess,
                                     torque_dev),
                       "right-hand side");
                loc.rhs_evals++;
                torque_known = false;
            } else {
                std::swap(k[0], k[6]);
            }
            double fac = err == 0.0 ? 10.0 : std::min(10.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
            if (last_rejected && fac > 1.0) fac = 1.0;
            if (!(h < *dt)) *dt = fac * h;
            last_rejected = false;
        } else {
            loc.rejected++;
            *dt = std::max(0.2, 0.9 * std::pow(err, -0.2)) * h;
            last_rejected = true;
        }
        if (*dt < dt_min) {
            set_error("step size fell below dt_min");
            status = MM_EDTMIN;
            break;
        }
    }
    if (relax && status == MM_OK) {
        if (!torque_known) {
            mm_status s2 = fetch(p, 2);
            if (s2 != MM_OK) return s2;
            torque = p->host_out[1];
        }
        if (!(torque < torque_tol)) {
            set_error("relaxation did not reach the torque criterion");
            status = MM_ENOTCONV;
        }
    }
    MM_HIP(hipMemcpyAsync(m_user, y, vbytes, hipMemcpyDeviceToDevice, p->stream), "copy m");
    MM_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
    loc.t = *t;
    loc.dt = *dt;
    if (st) *st = loc;
    return status;
}

// Allocate and set up a plan from validated arguments.  With `share`, the
// spectral kernel and twiddles of another plan of the same grid class are
// reused (reference counted) instead of built.
mm_status plan_build(const int grid[3], const double cell[3], double Ms, double A, double Ku,
                     double alpha, const mm_opts& o, SharedTensor* share, Plan** out, int batch)
{
    *out = nullptr;
    if (batch < 1 || batch > 64 || (batch > 1 && (o.workspace || o.dz_layers))) {
        set_error("a batch plan holds 1 to 64 equal-layer requests and no caller workspace");
        return MM_EINVAL;
    }
    const double nrm = std::sqrt(o.ku_axis[0] * o.ku_axis[0] + o.ku_axis[1] * o.ku_axis[1] +
                                 o.ku_axis[2] * o.ku_axis[2]);
    Plan* p = new Plan();
    for (int a = 0; a < 3; ++a) {
        p->n[a] = grid[a];
        p->d[a] = cell[a];
        p->P[a] = padded_extent(grid[a]);
        p->eu[a] = o.ku_axis[a] / nrm;
    }
    p->N = (long)grid[0] * grid[1] * grid[2];
    if (o.dz_layers && grid[2] > 1) {
        // thin layers of unequal height: no z padding, dense layer coupling
        p->layered = true;
        p->P[2] = 1;
        p->zb.assign(grid[2] + 1, 0.0);
        for (int k = 0; k < grid[2]; ++k) p->zb[k + 1] = p->zb[k] + o.dz_layers[k];
        p->d[2] = o.dz_layers[0];
    }
    p->Hx = p->P[0] > 1 ? p->P[0] / 2 + 1 : 1;
    // spectral rows start on 128-byte boundaries for the real kernel array
    // (32 floats or 16 doubles) and therefore for the complex spectra too
    const int row_align = o.prec == MM_FP32 ? 32 : 16;
    p->Hxp = (p->Hx + row_align - 1) / row_align * row_align;
    p->S1n = 3L * grid[2] * grid[1] * p->Hxp;
    p->S2n = 3L * grid[2] * p->P[1] * p->Hxp;
    // layered: one kernel per unordered layer pair, nz (nz + 1) / 2 of them
    p->Kn = p->layered ? (long)grid[2] * (grid[2] + 1) / 2 * (p->P[1] / 2 + 1) * p->Hxp
                       : (long)(p->P[2] / 2 + 1) * (p->P[1] / 2 + 1) * p->Hxp;
    p->Lmax = std::max(p->P[0], std::max(p->P[1], p->P[2]));
    p->prec = o.prec;
    p->Ms = Ms;
    p->A = A;
    p->Ku = Ku;
    p->alpha = alpha;
    p->Ku2 = o.ku2;
    p->Kc1 = o.kc1;
    p->Kc2 = o.kc2;
    {
        // cubic axes: c1 normalised, c2 made orthogonal to it, c3 = c1 x c2
        double a1[3], a2[3];
        const double n1 = std::sqrt(o.kc_axis1[0] * o.kc_axis1[0] + o.kc_axis1[1] * o.kc_axis1[1] +
                                    o.kc_axis1[2] * o.kc_axis1[2]);
        for (int a = 0; a < 3; ++a) a1[a] = o.kc_axis1[a] / n1;
        const double pr = o.kc_axis2[0] * a1[0] + o.kc_axis2[1] * a1[1] + o.kc_axis2[2] * a1[2];
        double n2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            a2[a] = o.kc_axis2[a] - pr * a1[a];
            n2 += a2[a] * a2[a];
        }
        n2 = std::sqrt(n2);
        for (int a = 0; a < 3; ++a) {
            p->ec[0][a] = a1[a];
            p->ec[1][a] = a2[a] / n2;
        }
        p->ec[2][0] = p->ec[0][1] * p->ec[1][2] - p->ec[0][2] * p->ec[1][1];
        p->ec[2][1] = p->ec[0][2] * p->ec[1][0] - p->ec[0][0] * p->ec[1][2];
        p->ec[2][2] = p->ec[0][0] * p->ec[1][1] - p->ec[0][1] * p->ec[1][0];
    }
    p->demag_p = o.demag_p;
    p->percell = false;
    p->percell_A = p->percell_D = p->dmi = p->dmi_mixed = false;
    p->dmi_type = MM_DMI_INTERFACE;
    p->D = 0.0;
    std::memset(p->edmi, 0, sizeof(p->edmi));
    p->n_magnetic = Ms > 0.0 ? p->N : 0;
    p->drive = false;
    p->stream = (hipStream_t)o.stream;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            ncu > 0)
            p->ncu = ncu;
    }
    const size_t es = elem_size(*p);
    mm_status s;
    (void)s;
#define MM_ALLOC(ptr, bytes, what)                              \
    do {                                                        \
        s = alloc(p, (void**)&(ptr), (bytes), what);            \
        if (s != MM_OK) {                                       \
            free_plan(p);                                       \
            return s;                                           \
        }                                                       \
    } while (0)
    if (o.workspace) {
        // the caller's workspace holds every persistent buffer (checked by
        // mm_plan_create: equal layers, large enough, 256-byte aligned)
        const WsLayout L = ws_layout(grid, o.prec);
        char* w = static_cast<char*>(o.workspace);
        p->ws = true;
        p->Khat = w + L.Khat;
        p->S1 = w + L.S1;
        p->S2 = L.s2_separate ? (void*)(w + L.S2) : p->S1;
        p->tw = w + L.tw;
        p->red = reinterpret_cast<double*>(w + L.red);
        p->red_out = reinterpret_cast<double*>(w + L.red_out);
        p->rk = w + L.rk;
        p->ctl = reinterpret_cast<DevCtl*>(w + L.ctl);
        p->epart = reinterpret_cast<double*>(w + L.epart);
        p->bytes = L.total;
    } else {
    // a batch plan: spectra, reductions and controllers for every request
    const size_t nb = (size_t)batch;
    p->batch = batch;
    p->vstride = batch > 1 ? 3 * p->N * batch : 0;
    if (!share) MM_ALLOC(p->Khat, 6 * (size_t)p->Kn * es, "spectral kernel");
    MM_ALLOC(p->S1, (size_t)p->S1n * 2 * es * nb, "spectrum S1");
    if ((p->P[2] > 1 || p->layered) && p->P[1] > 1)
        MM_ALLOC(p->S2, (size_t)p->S2n * 2 * es * nb, "spectrum S2");
    else
        p->S2 = p->S1;
    if (!share) MM_ALLOC(p->tw, (size_t)p->Lmax * 2 * es, "twiddles");
    MM_ALLOC(p->red, sizeof(double) * kRedSlots * nb, "reduction partials");
    MM_ALLOC(p->red_out, sizeof(double) * 8 * nb, "reduction results");
    if (batch > 1) {
        MM_ALLOC(p->Pb, (batch_slot_bytes() - sizeof(double)) * nb, "per-request constants");
        MM_ALLOC(p->Ms_b, es * nb, "per-request Ms");
        hipError_t eh = hipHostMalloc(&p->Pb_host, batch_slot_bytes() * nb, hipHostMallocDefault);
        if (eh != hipSuccess) {
            p->Pb_host = nullptr;
            free_plan(p);
            return hip_fail(eh, "per-request constants staging");
        }
    }
    }
    if (p->layered) {
        MM_ALLOC(p->zw, 4 * (size_t)grid[2] * es, "layer couplings");
        MM_ALLOC(p->lw, sizeof(double) * grid[2], "layer heights");
    }
#undef MM_ALLOC
    if (p->layered) {
        // z exchange to the layer below / above, 2/(dz_k (dz_k + dz_j)) (the
        // flux between the centres per height of the layer), and 1/(2 dz_k)
        // for the DMI difference; heights for the energies
        const int nz = grid[2];
        std::vector<double> zw(4 * nz, 0.0), lw(nz);
        for (int k = 0; k < nz; ++k) {
            const double hk = p->zb[k + 1] - p->zb[k];
            lw[k] = hk;
            if (k > 0) zw[4 * k] = 2.0 / (hk * (hk + (p->zb[k] - p->zb[k - 1])));
            if (k + 1 < nz) zw[4 * k + 1] = 2.0 / (hk * (hk + (p->zb[k + 2] - p->zb[k + 1])));
            zw[4 * k + 2] = 1.0 / (2.0 * hk);
        }
        hipError_t e1 = hipSuccess;
        if (p->prec == MM_FP32) {
            std::vector<float> zf(zw.begin(), zw.end());
            e1 = hipMemcpy(p->zw, zf.data(), sizeof(float) * zf.size(), hipMemcpyHostToDevice);
        } else {
            e1 = hipMemcpy(p->zw, zw.data(), sizeof(double) * zw.size(), hipMemcpyHostToDevice);
        }
        if (e1 == hipSuccess)
            e1 = hipMemcpy(p->lw, lw.data(), sizeof(double) * nz, hipMemcpyHostToDevice);
        if (e1 != hipSuccess) {
            free_plan(p);
            return hip_fail(e1, "layer tables");
        }
    }
    hipError_t e = hipHostMalloc((void**)&p->host_out, sizeof(double) * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "pinned host buffer");
    }
    if (share) {
        p->Khat = share->Khat;
        p->tw = share->tw;
        p->shared = share;
        share->refs++;
        *out = p;
        return MM_OK;
    }
    e = p->prec == MM_FP32 ? init_twiddles<float>(*p) : init_twiddles<double>(*p);
    if (e == hipSuccess) e = p->prec == MM_FP32 ? build_tensor<float>(*p) : build_tensor<double>(*p);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        mm_status st = hip_fail(e, "building the demag kernel");
        free_plan(p);
        return st;
    }
    *out = p;
    return MM_OK;
}


// Layout of a plan's persistent buffers in one workspace; mirrors the
// allocations of plan_build and ensure_rk (equal layers).
WsLayout ws_layout(const int grid[3], int prec)
{
    const size_t es = prec == MM_FP32 ? 4 : 8;
    int P[3];
    for (int a = 0; a < 3; ++a) P[a] = padded_extent(grid[a]);
    const long N = (long)grid[0] * grid[1] * grid[2];
    const int Hx = P[0] > 1 ? P[0] / 2 + 1 : 1;
    const int row_align = prec == MM_FP32 ? 32 : 16;
    const long Hxp = (Hx + row_align - 1) / row_align * row_align;
    const long S1n = 3L * grid[2] * grid[1] * Hxp;
    const long S2n = 3L * grid[2] * P[1] * Hxp;
    const long Kn = (long)(P[2] / 2 + 1) * (P[1] / 2 + 1) * Hxp;
    const int Lmax = std::max(P[0], std::max(P[1], P[2]));
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    WsLayout L{};
    size_t off = 0;
    L.Khat = off;
    off += up(6 * (size_t)Kn * es);
    L.S1 = off;
    off += up((size_t)S1n * 2 * es);
    L.s2_separate = P[2] > 1 && P[1] > 1;
    L.S2 = off;
    if (L.s2_separate) off += up((size_t)S2n * 2 * es);
    L.tw = off;
    off += up((size_t)Lmax * 2 * es);
    L.red = off;
    off += up(sizeof(double) * kRedSlots);
    L.red_out = off;
    off += up(sizeof(double) * 8);
    L.rk = off;
    off += up(10 * 3 * (size_t)N * es);
    L.ctl = off;
    off += up(sizeof(DevCtl));
    L.epart = off;
    off += up(2 * sizeof(double) * (size_t)grid[1] * grid[2]);
    L.total = off;
    return L;
}

// Device bytes a plan of this grid allocates for a device-controlled run
// (spectra, reduction buffers, Runge-Kutta vectors, controller), plus the
// spectral kernel and twiddles when with_tensor.
size_t plan_footprint(const int grid[3], int prec, bool with_tensor)
{
    const WsLayout L = ws_layout(grid, prec);
    return with_tensor ? L.total : L.total - (L.S1 - L.Khat) - (L.red - L.tw);
}

size_t batch_footprint(const int grid[3], int prec, int batch, bool state64)
{
    // per request: the spectra, reductions, Runge-Kutta space and controller
    // of a plan without kernel, the double state, its constants; rounding
    // to 256 bytes per buffer is counted once per request (an upper bound)
    const size_t es = prec == MM_FP32 ? 4 : 8;
    const size_t per = plan_footprint(grid, prec, false) + (state64 ? state64_bytes(grid) : 0) +
                       (batch > 1 ? batch_slot_bytes() + es : 0);
    return per * (size_t)batch;
}

Plan batch_view(const Plan& g, int b)
{
    Plan v = g;
    const size_t es = elem_size(g);
    const long n3 = 3 * g.N;
    v.batch = 1;
    v.Pb = v.Ms_b = v.Pb_host = nullptr;
    v.shared = nullptr;
    v.ws = true;  // owns nothing
    v.S1 = static_cast<char*>(g.S1) + (size_t)b * g.S1n * 2 * es;
    v.S2 = g.S2 == g.S1 ? v.S1 : static_cast<char*>(g.S2) + (size_t)b * g.S2n * 2 * es;
    v.red = g.red + (size_t)b * kRedSlots;
    v.red_out = g.red_out + (size_t)b * 8;
    v.rk = g.rk ? static_cast<char*>(g.rk) + (size_t)b * n3 * es : nullptr;
    v.vstride = n3 * g.batch;
    v.st64 = g.st64 ? g.st64 + (size_t)b * n3 : nullptr;
    v.ctl = g.ctl ? g.ctl + b : nullptr;
    v.prof = Profiler{};
    return v;
}

}  // namespace mmx

using namespace mmx;

namespace mmx {

// Adjoint work-space layout (vectors of 3N): 0 y, 1 ynew, 2 ys, 3-6 k1..k4,
// 7 z, 8 g, 9 lambda, 10 kappa, 11-14 nu1..nu4, 15 field scratch.
template <typename T>
static mm_status rk4_step_impl(Plan* p, T* y, T* ynew, const double hext[3], unsigned terms,
                               double t, double dt, T* const* ys_store, T* const* hs_store)
{
    T* k[4] = {adj_vec<T>(p, 3), adj_vec<T>(p, 4), adj_vec<T>(p, 5), adj_vec<T>(p, 6)};
    T* ys = adj_vec<T>(p, 2);
    const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    const double half = 0.5, one = 1.0;
    for (int st = 0; st < 4; ++st) {
        const T* in = y;
        if (st > 0) {
            T* prev = k[st - 1];
            MM_HIP(rk_combine<T>(*p, ys, y, dt, st == 3 ? &one : &half, &prev, 1), "stage input");
            in = ys;
        }
        if (ys_store)
            MM_HIP(hipMemcpyAsync(ys_store[st], in, 3 * (size_t)p->N * sizeof(T),
                                  hipMemcpyDeviceToDevice, p->stream),
                   "store stage");
        MM_HIP(eval_field<T>(*p, in, hext, terms, t + cs[st] * dt, hs_store ? hs_store[st] : nullptr,
                             k[st], p->alpha, true, nullptr),
               "right-hand side");
    }
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    MM_HIP(rk_combine<T>(*p, ynew, y, dt, b, k, 4), "RK4 update");
    return MM_OK;
}

// number of cells in a region mask: the region sum of m_z for a vector whose
// z component is one on the region and zero elsewhere
template <typename T>
static mm_status count_region(Plan* p, const unsigned char* region, long* nreg)
{
    T* ind = adj_vec<T>(p, 15);
    MM_HIP(hipMemsetAsync(ind, 0, 3 * (size_t)p->N * sizeof(T), p->stream), "clear");
    MM_HIP(add_region<T>(*p, ind, region, 1.0), "region indicator");
    MM_HIP(hipMemsetAsync(p->red_out + 7, 0, sizeof(double), p->stream), "clear");
    MM_HIP(region_mz_accum<T>(*p, ind, region, p->red_out + 7, 1.0), "count region");
    mm_status s = fetch(p, 8);
    if (s != MM_OK) return s;
    *nreg = (long)std::llround(p->host_out[7]);
    return MM_OK;
}

template <typename T>
static mm_status rk4_forward_impl(Plan* p, void* m_user, const double hext[3], unsigned terms,
                                  double t0, double dt, long nsteps, const unsigned char* region,
                                  long every, void* ckpt, double* loss)
{
    mm_status s = ensure_adj(p);
    if (s != MM_OK) return s;
    const size_t vb = 3 * (size_t)p->N * sizeof(T);
    long nreg = 0;
    if (region) {
        s = count_region<T>(p, region, &nreg);
        if (s != MM_OK) return s;
    }
    T* y = adj_vec<T>(p, 0);
    T* ynew = adj_vec<T>(p, 1);
    MM_HIP(hipMemcpyAsync(y, m_user, vb, hipMemcpyDeviceToDevice, p->stream), "copy m");
    MM_HIP(hipMemsetAsync(p->red_out + 6, 0, sizeof(double), p->stream), "clear loss");
    for (long n = 0; n < nsteps; ++n) {
        if (ckpt && every > 0 && n % every == 0)
            MM_HIP(hipMemcpyAsync((T*)ckpt + (size_t)(n / every) * 3 * p->N, y, vb,
                                  hipMemcpyDeviceToDevice, p->stream),
                   "checkpoint");
        s = rk4_step_impl<T>(p, y, ynew, hext, terms, t0 + n * dt, dt, nullptr, nullptr);
        if (s != MM_OK) return s;
        std::swap(y, ynew);
        if (region && nreg > 0) MM_HIP(region_mz_accum<T>(*p, y, region, p->red_out + 6, 1.0), "loss");
    }
    MM_HIP(hipMemcpyAsync(m_user, y, vb, hipMemcpyDeviceToDevice, p->stream), "copy m");
    s = fetch(p, 7);
    if (s != MM_OK) return s;
    if (loss) *loss = (region && nreg > 0 && nsteps > 0) ? p->host_out[6] / ((double)nsteps * nreg) : 0.0;
    return MM_OK;
}

template <typename T>
static mm_status rk4_adjoint_impl(Plan* p, const void* ckpt, const double hext[3], unsigned terms,
                                  double t0, double dt, long nsteps, const unsigned char* region,
                                  long every, void* grad_ms, void* grad_m0, double* loss)
{
    mm_status s = ensure_adj(p);
    if (s != MM_OK) return s;
    const size_t vb = 3 * (size_t)p->N * sizeof(T);
    const size_t need = (size_t)every * 8 * vb;
    if (p->seg_bytes < need) {
        if (p->seg) {
            (void)hipFree(p->seg);
            p->bytes -= p->seg_bytes;
            p->seg = nullptr;
            p->seg_bytes = 0;
        }
        s = alloc(p, &p->seg, need, "checkpoint segment");
        if (s != MM_OK) return s;
        p->seg_bytes = need;
    }
    long nreg = 0;
    s = count_region<T>(p, region, &nreg);
    if (s != MM_OK) return s;
    const double dL = nreg > 0 ? 1.0 / ((double)nsteps * nreg) : 0.0;
    const unsigned vterms = terms & ~(unsigned)(MM_ZEEMAN | MM_OERSTED);
    T* y = adj_vec<T>(p, 0);
    T* ynew = adj_vec<T>(p, 1);
    T* z = adj_vec<T>(p, 7);
    T* g = adj_vec<T>(p, 8);
    T* lam = adj_vec<T>(p, 9);
    T* kap = adj_vec<T>(p, 10);
    T* nu[4] = {adj_vec<T>(p, 11), adj_vec<T>(p, 12), adj_vec<T>(p, 13), adj_vec<T>(p, 14)};
    MM_HIP(hipMemsetAsync(lam, 0, vb, p->stream), "clear lambda");
    MM_HIP(zero_doubles(*p, p->gms, p->N), "clear gradient");
    MM_HIP(hipMemsetAsync(p->red_out + 6, 0, sizeof(double), p->stream), "clear loss");
    const long nseg = (nsteps + every - 1) / every;
    auto Ys = [&](long i, int st) { return (T*)p->seg + ((size_t)i * 8 + st) * 3 * p->N; };
    auto Hs = [&](long i, int st) { return (T*)p->seg + ((size_t)i * 8 + 4 + st) * 3 * p->N; };
    for (long sg = nseg - 1; sg >= 0; --sg) {
        const long n0 = sg * every, n1 = std::min(nsteps, n0 + every);
        MM_HIP(hipMemcpyAsync(y, (const T*)ckpt + (size_t)sg * 3 * p->N, vb,
                              hipMemcpyDeviceToDevice, p->stream),
               "restore checkpoint");
        for (long n = n0; n < n1; ++n) {
            T* ysv[4] = {Ys(n - n0, 0), Ys(n - n0, 1), Ys(n - n0, 2), Ys(n - n0, 3)};
            T* hsv[4] = {Hs(n - n0, 0), Hs(n - n0, 1), Hs(n - n0, 2), Hs(n - n0, 3)};
            s = rk4_step_impl<T>(p, y, ynew, hext, terms, t0 + n * dt, dt, ysv, hsv);
            if (s != MM_OK) return s;
            std::swap(y, ynew);
            MM_HIP(region_mz_accum<T>(*p, y, region, p->red_out + 6, 1.0), "loss");
        }
        for (long n = n1 - 1; n >= n0; --n) {
            const long i = n - n0;
            MM_HIP(add_region<T>(*p, lam, region, dL), "loss gradient");
            // kappa_4 = dt/6 lam;  kappa_3 = dt/3 lam + dt nu_4;
            // kappa_2 = dt/3 lam + dt/2 nu_3;  kappa_1 = dt/6 lam + dt/2 nu_2
            const double cl[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
            const double cn[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
            for (int st = 3; st >= 0; --st) {
                if (st == 3) {
                    T* v1[1] = {lam};
                    MM_HIP(lincomb<T>(*p, kap, &cl[3], v1, 1), "cotangent");
                } else {
                    T* v2[2] = {lam, nu[st + 1]};
                    const double c2[2] = {cl[st], cn[st + 1]};
                    MM_HIP(lincomb<T>(*p, kap, c2, v2, 2), "cotangent");
                }
                MM_HIP(field_vjp<T>(*p, Ys(i, st), kap, Hs(i, st), vterms, p->alpha, g, z, nu[st],
                                    p->gms),
                       "vector-Jacobian product");
            }
            T* v5[5] = {lam, nu[0], nu[1], nu[2], nu[3]};
            const double c5[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
            MM_HIP(lincomb<T>(*p, lam, c5, v5, 5), "adjoint update");
        }
    }
    if (grad_m0)
        MM_HIP(hipMemcpyAsync(grad_m0, lam, vb, hipMemcpyDeviceToDevice, p->stream), "grad m0");
    if (grad_ms) MM_HIP(from_double<T>(*p, p->gms, (T*)grad_ms, p->N), "grad Ms");
    s = fetch(p, 7);
    if (s != MM_OK) return s;
    if (loss) *loss = nreg > 0 ? p->host_out[6] / ((double)nsteps * nreg) : 0.0;
    return MM_OK;
}

static bool nonlinear_anis(const Plan* p, unsigned terms)
{
    return (terms & MM_ANIS) && (p->Ku2 != 0.0 || p->Kc1 != 0.0 || p->Kc2 != 0.0);
}

// The transposed operators cover the uniform-A exchange stencil and the
// uniform uniaxial constant only.
static bool stencil_extended(const Plan* p, unsigned terms)
{
    return ((terms & MM_EXCH) && p->percell_A) || ((terms & MM_DMI) && p->dmi) ||
           ((terms & MM_ANIS) && p->percell_Ku);
}

template <typename T>
static mm_status heff_vjp_impl(Plan* p, const T* m, const T* w, const double hext[3],
                               unsigned terms, double t, bool llg, T* grad_m, T* grad_ms)
{
    if (nonlinear_anis(p, terms)) {
        set_error("higher-order anisotropy is not linear in m: no transposed operator");
        return MM_EINVAL;
    }
    if (stencil_extended(p, terms)) {
        set_error("per-cell exchange, per-cell Ku and DMI have no transposed operator");
        return MM_EINVAL;
    }
    if (p->layered) {
        set_error("thin layers of unequal height have no transposed operator");
        return MM_EINVAL;
    }
    mm_status s = ensure_adj(p);
    if (s != MM_OK) return s;
    T* h = nullptr;
    if (llg) {
        h = adj_vec<T>(p, 15);
        MM_HIP(eval_field<T>(*p, m, hext, terms, t, h, nullptr, p->alpha, true, nullptr), "field");
    }
    MM_HIP(zero_doubles(*p, p->gms, p->N), "clear gradient");
    MM_HIP(field_vjp<T>(*p, m, w, h, terms & ~(unsigned)(MM_ZEEMAN | MM_OERSTED), p->alpha,
                        adj_vec<T>(p, 8),
                        adj_vec<T>(p, 7), grad_m, p->gms),
           "vector-Jacobian product");
    if (grad_ms) MM_HIP(from_double<T>(*p, p->gms, grad_ms, p->N), "grad Ms");
    return MM_OK;
}

// The energies of `terms` at m into E[6]: the field of each term into h (3N
// reals), its weighted dot product with m reduced through `partials`
// (kRedSlots doubles) into out[0..4], read back through the plan's pinned
// buffer.  Every slot of out is written (cleared by a fill kernel, not a
// memset, so the sequence can sit in a captured graph).  Synchronises.
template <typename T>
static mm_status energy_core(Plan* p, const T* m, const double h_ext[3], unsigned terms, double t,
                             T* h, double* partials, double* out, double E[6])
{
    // reduction slots 0..3 demag, exchange, anisotropy, Zeeman (with the
    // Oersted field, an applied field too); 4 DMI
    const unsigned bits[5] = {MM_DEMAG, MM_EXCH, MM_ANIS, MM_ZEEMAN | MM_OERSTED, MM_DMI};
    MM_HIP(zero_doubles(*p, out, 8), "clear");
    for (int e = 0; e < 5; ++e) {
        if (!(terms & bits[e])) continue;
        if (bits[e] == MM_ANIS) {
            // from the energy density (the linear-term formula does not hold
            // for the higher orders)
            MM_HIP(anis_energy<T>(*p, m, out + e, partials), "anisotropy energy");
            continue;
        }
        MM_HIP(eval_field<T>(*p, m, h_ext, bits[e] & terms, t, h, nullptr, p->alpha, true, nullptr),
               "field");
        MM_HIP(dot_ms<T>(*p, m, h, out + e, partials), "energy reduction");
    }
    MM_HIP(hipMemcpyAsync(p->host_out, out, sizeof(double) * 5, hipMemcpyDeviceToHost, p->stream),
           "reading a reduction");
    MM_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
    // thin layers: the reductions carry each layer's height
    const double V = p->d[0] * p->d[1] * (p->layered ? 1.0 : p->d[2]);
    double tot = 0.0;
    for (int e = 0; e < 4; ++e) {
        E[e] = e == 2 ? V * p->host_out[e] : (e == 3 ? -1.0 : -0.5) * kMu0 * V * p->host_out[e];
        tot += E[e];
    }
    // the DMI operator is symmetric in the Ms-weighted product, so the
    // linear-term formula holds
    E[5] = -0.5 * kMu0 * V * p->host_out[4];
    E[4] = tot + E[5];
    return MM_OK;
}

template <typename T>
static mm_status energy_impl(Plan* p, const T* m, const double h_ext[3], unsigned terms, double t,
                             double E[6])
{
    mm_status s = ensure_rk(p);
    if (s != MM_OK) return s;
    return energy_core<T>(p, m, h_ext, terms, t, rk_vec<T>(p, 0), p->red, p->red_out, E);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (mm_energy_noalloc): one static
// device array per GPU, held until the process ends.  Host code never passes
// the array's name to a kernel or copy; it uses the device address that
// hipGetSymbolAddress returns, fetched once per device on the first call made
// with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static mm_status scratch_address(void** out)
{
    int dev = 0;
    MM_HIP(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the scratch table");
        return MM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        MM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MM_OK;
}

// Scratch layout: reduction partials (kRedSlots doubles), results (8
// doubles, padded to 256 bytes), then the field buffer of 3N reals.
constexpr size_t kScratchPartials = 0;
constexpr size_t kScratchOut = sizeof(double) * kRedSlots;
constexpr size_t kScratchField = kScratchOut + 256;

template <typename T>
static mm_status energy_noalloc_impl(Plan* p, const T* m, const double h_ext[3], unsigned terms,
                                     double t, double E[6])
{
    const size_t need = kScratchField + 3 * (size_t)p->N * sizeof(T);
    if (need > (size_t)MM_NOALLOC_SCRATCH_BYTES) {
        set_error("mm_energy_noalloc: the plan needs " + std::to_string(need) +
                  " bytes of scratch, the maximum is " + std::to_string((size_t)MM_NOALLOC_SCRATCH_BYTES));
        return MM_EINVAL;
    }
    void* base = nullptr;
    mm_status s = scratch_address(&base);
    if (s != MM_OK) return s;
    char* b = static_cast<char*>(base);
    return energy_core<T>(p, m, h_ext, terms, t, reinterpret_cast<T*>(b + kScratchField),
                          reinterpret_cast<double*>(b + kScratchPartials),
                          reinterpret_cast<double*>(b + kScratchOut), E);
}

}  // namespace mmx

extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

void mm_opts_default(mm_opts* o)
{
    if (!o) return;
    o->prec = MM_FP64;
    o->ku_axis[0] = 0.0;
    o->ku_axis[1] = 0.0;
    o->ku_axis[2] = 1.0;
    o->demag_p = 20;
    o->stream = nullptr;
    o->ku2 = o->kc1 = o->kc2 = 0.0;
    o->dz_layers = nullptr;
    o->workspace = nullptr;
    o->workspace_bytes = 0;
    for (int a = 0; a < 3; ++a) {
        o->kc_axis1[a] = a == 0 ? 1.0 : 0.0;
        o->kc_axis2[a] = a == 1 ? 1.0 : 0.0;
    }
}

mm_status mm_plan_create(mm_plan** out, const int grid[3], const double cell[3], double Ms,
                         double A, double Ku, double alpha, const mm_opts* opt)
{
    if (!out || !grid || !cell) {
        set_error("null argument");
        return MM_EINVAL;
    }
    *out = nullptr;
    mm_opts o;
    mm_opts_default(&o);
    if (opt) o = *opt;
    for (int a = 0; a < 3; ++a) {
        if (grid[a] < 1 || grid[a] > kMaxFFT / 2) {
            set_error("grid extents must lie in [1, 512]");
            return MM_EINVAL;
        }
        if (!(cell[a] > 0.0) || !std::isfinite(cell[a])) {
            set_error("cell sizes must be positive and finite");
            return MM_EINVAL;
        }
    }
    if (!(Ms >= 0.0) || !(A >= 0.0) || !(alpha >= 0.0) || !std::isfinite(Ms) || !std::isfinite(A) ||
        !std::isfinite(Ku) || !std::isfinite(alpha)) {
        set_error("Ms, A and alpha must be finite and non-negative, Ku finite");
        return MM_EINVAL;
    }
    if (o.prec != MM_FP32 && o.prec != MM_FP64) {
        set_error("precision must be MM_FP32 or MM_FP64");
        return MM_EINVAL;
    }
    const double nrm = std::sqrt(o.ku_axis[0] * o.ku_axis[0] + o.ku_axis[1] * o.ku_axis[1] +
                                 o.ku_axis[2] * o.ku_axis[2]);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) {
        set_error("anisotropy axis must be a non-zero finite vector");
        return MM_EINVAL;
    }
    {
        const double* c1 = o.kc_axis1;
        const double* c2 = o.kc_axis2;
        const double n1 = std::sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
        const double cx = c1[1] * c2[2] - c1[2] * c2[1], cy = c1[2] * c2[0] - c1[0] * c2[2],
                     cz = c1[0] * c2[1] - c1[1] * c2[0];
        if (!std::isfinite(o.ku2) || !std::isfinite(o.kc1) || !std::isfinite(o.kc2) ||
            !(n1 > 0.0) || !(cx * cx + cy * cy + cz * cz > 0.0) || !std::isfinite(cx + cy + cz)) {
            set_error("ku2, kc1, kc2 must be finite and the cubic axes independent");
            return MM_EINVAL;
        }
    }
    if (o.dz_layers) {
        if (grid[2] > kMaxLayers) {
            set_error("thin layers: at most 16 layers");
            return MM_EINVAL;
        }
        for (int k = 0; k < grid[2]; ++k)
            if (!(o.dz_layers[k] > 0.0) || !std::isfinite(o.dz_layers[k])) {
                set_error("layer heights must be positive and finite");
                return MM_EINVAL;
            }
    }
    if (o.workspace) {
        const size_t need = ws_layout(grid, o.prec).total;
        if (o.dz_layers) {
            set_error("a caller workspace holds equal-layer plans only");
            return MM_EINVAL;
        }
        if (((uintptr_t)o.workspace & 255) != 0) {
            set_error("the workspace must be aligned to 256 bytes");
            return MM_EINVAL;
        }
        if (o.workspace_bytes < need) {
            set_error("workspace of " + std::to_string(o.workspace_bytes) + " bytes, " +
                      std::to_string(need) + " needed (mm_plan_workspace_bytes)");
            return MM_EINVAL;
        }
    }
    Plan* p = nullptr;
    mm_status s = plan_build(grid, cell, Ms, A, Ku, alpha, o, nullptr, &p);
    if (s != MM_OK) return s;
    *out = reinterpret_cast<mm_plan*>(p);
    return MM_OK;
}

size_t mm_plan_workspace_bytes(const int grid[3], int prec)
{
    if (!grid || (prec != MM_FP32 && prec != MM_FP64)) return 0;
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1 || grid[a] > kMaxFFT / 2) return 0;
    return ws_layout(grid, prec).total;
}

void mm_plan_destroy(mm_plan* pl) { free_plan(reinterpret_cast<Plan*>(pl)); }

size_t mm_plan_device_bytes(const mm_plan* pl)
{
    return pl ? reinterpret_cast<const Plan*>(pl)->bytes : 0;
}

void mm_plan_padded(const mm_plan* pl, int P[3])
{
    const Plan* p = reinterpret_cast<const Plan*>(pl);
    for (int a = 0; a < 3; ++a) P[a] = p ? p->P[a] : 0;
}

mm_status mm_set_ms(mm_plan* pl, const void* Ms_cell)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    if (!Ms_cell) {
        p->percell = false;
        p->n_magnetic = p->Ms > 0.0 ? p->N : 0;
        return MM_OK;
    }
    const size_t bytes = (size_t)p->N * elem_size(*p);
    if (!p->Ms_cell) {
        mm_status s = alloc(p, &p->Ms_cell, bytes, "per-cell Ms");
        if (s != MM_OK) return s;
    }
    MM_HIP(hipMemcpyAsync(p->Ms_cell, Ms_cell, bytes, hipMemcpyDeviceToDevice, p->stream),
           "copy Ms");
    p->percell = true;
    MM_HIP(p->prec == MM_FP32 ? count_magnetic<float>(*p, p->red_out)
                              : count_magnetic<double>(*p, p->red_out),
           "count magnetic cells");
    mm_status s = fetch(p, 1);
    if (s != MM_OK) return s;
    p->n_magnetic = (long)std::llround(p->host_out[0]);
    return MM_OK;
}

// Copy N values of the plan's precision into *dst (allocated on first use).
static mm_status copy_cell_field(Plan* p, void** dst, const void* src, const char* what)
{
    const size_t bytes = (size_t)p->N * elem_size(*p);
    if (!*dst) {
        mm_status s = alloc(p, dst, bytes, what);
        if (s != MM_OK) return s;
    }
    MM_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyDeviceToDevice, p->stream), what);
    return MM_OK;
}

mm_status mm_set_exchange(mm_plan* pl, const void* A_cell)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    if (!A_cell) {
        p->percell_A = false;
        return MM_OK;
    }
    mm_status s = copy_cell_field(p, &p->A_cell, A_cell, "per-cell exchange constant");
    if (s != MM_OK) return s;
    p->percell_A = true;
    return MM_OK;
}

mm_status mm_set_ku(mm_plan* pl, const void* Ku_cell)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    if (!Ku_cell) {
        p->percell_Ku = false;
        return MM_OK;
    }
    mm_status s = copy_cell_field(p, &p->Ku_cell, Ku_cell, "per-cell uniaxial constant");
    if (s != MM_OK) return s;
    p->percell_Ku = true;
    return MM_OK;
}

mm_status mm_set_dmi(mm_plan* pl, int type, double D, const void* D_cell)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    if (type < MM_DMI_INTERFACE || type > MM_DMI_D2D || !std::isfinite(D)) {
        set_error("invalid DMI type or strength");
        return MM_EINVAL;
    }
    p->dmi_mixed = false;
    if (D_cell) {
        mm_status s = copy_cell_field(p, &p->D_cell, D_cell, "per-cell DMI strength");
        if (s != MM_OK) return s;
        // opposite-sign neighbour pairs need the second case of Eq. D_avg
        MM_HIP(p->prec == MM_FP32 ? count_signs<float>(*p, (const float*)p->D_cell, p->red_out)
                                  : count_signs<double>(*p, (const double*)p->D_cell, p->red_out),
               "DMI signs");
        s = fetch(p, 2);
        if (s != MM_OK) return s;
        p->dmi_mixed = p->host_out[0] > 0.0 && p->host_out[1] > 0.0;
    }
    p->percell_D = D_cell != nullptr;
    p->D = D_cell ? 0.0 : D;
    p->dmi = D_cell != nullptr || D != 0.0;
    p->dmi_type = type;
    // DMI vectors (e^dmi_x, e^dmi_y, e^dmi_z) of the tabulated types
    std::memset(p->edmi, 0, sizeof(p->edmi));
    if (type == MM_DMI_INTERFACE) {
        p->edmi[0][1] = 1.0;   // e_y
        p->edmi[1][0] = -1.0;  // -e_x
    } else if (type == MM_DMI_BULK) {
        p->edmi[0][0] = p->edmi[1][1] = p->edmi[2][2] = 1.0;
    } else {
        p->edmi[0][0] = -1.0;  // -e_x
        p->edmi[1][1] = 1.0;   // e_y
    }
    return MM_OK;
}

mm_status mm_oersted(mm_plan* pl, const void* j, void* h_out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !j || !h_out || j == h_out) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    if (p->layered) {
        set_error("the Oersted kernel needs equal layers");
        return MM_EINVAL;
    }
    hipError_t e = p->prec == MM_FP32 ? oersted_field<float>(*p, (const float*)j, (float*)h_out)
                                      : oersted_field<double>(*p, (const double*)j, (double*)h_out);
    if (e != hipSuccess) return hip_fail(e, "Oersted field");
    return MM_OK;
}

mm_status mm_set_current(mm_plan* pl, const void* j, double freq)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !std::isfinite(freq)) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    if (!j) {
        p->oe_on = false;
        p->oe_freq = 0.0;
        return MM_OK;
    }
    if (p->layered) {
        set_error("the Oersted kernel needs equal layers");
        return MM_EINVAL;
    }
    if (!p->h_oe) {
        mm_status s = alloc(p, &p->h_oe, 3 * (size_t)p->N * elem_size(*p), "Oersted field");
        if (s != MM_OK) return s;
    }
    hipError_t e = p->prec == MM_FP32 ? oersted_field<float>(*p, (const float*)j, (float*)p->h_oe)
                                      : oersted_field<double>(*p, (const double*)j,
                                                              (double*)p->h_oe);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "Oersted field");
    p->oe_on = true;
    p->oe_freq = freq;
    return MM_OK;
}

mm_status mm_set_drive(mm_plan* pl, const double amp[3], double freq, const unsigned char* mask)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    if (!mask) {
        p->drive = false;
        return MM_OK;
    }
    if (!amp || !std::isfinite(freq)) {
        set_error("drive needs an amplitude and a finite frequency");
        return MM_EINVAL;
    }
    if (!p->mask) {
        mm_status s = alloc(p, (void**)&p->mask, (size_t)p->N, "drive mask");
        if (s != MM_OK) return s;
    }
    MM_HIP(hipMemcpyAsync(p->mask, mask, (size_t)p->N, hipMemcpyDeviceToDevice, p->stream),
           "copy mask");
    for (int a = 0; a < 3; ++a) p->drive_amp[a] = amp[a];
    p->drive_freq = freq;
    p->drive = true;
    return MM_OK;
}

static mm_status check_field_args(Plan* p, const void* m, const void* out)
{
    if (!p || !m || !out) {
        set_error("null argument");
        return MM_EINVAL;
    }
    if (m == out) {
        set_error("input and output buffers must not alias");
        return MM_EINVAL;
    }
    return MM_OK;
}

mm_status mm_heff(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms, double t,
                  void* h_out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    mm_status s = check_field_args(p, m, h_out);
    if (s != MM_OK) return s;
    hipError_t e = p->prec == MM_FP32
                       ? eval_field<float>(*p, (const float*)m, h_ext, terms, t, (float*)h_out,
                                           nullptr, p->alpha, true, nullptr)
                       : eval_field<double>(*p, (const double*)m, h_ext, terms, t,
                                            (double*)h_out, nullptr, p->alpha, true, nullptr);
    if (e != hipSuccess) return hip_fail(e, "mm_heff");
    return MM_OK;
}

mm_status mm_llg_rhs(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms, double t,
                     void* dmdt_out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    mm_status s = check_field_args(p, m, dmdt_out);
    if (s != MM_OK) return s;
    hipError_t e = p->prec == MM_FP32
                       ? eval_field<float>(*p, (const float*)m, h_ext, terms, t, nullptr,
                                           (float*)dmdt_out, p->alpha, true, nullptr)
                       : eval_field<double>(*p, (const double*)m, h_ext, terms, t, nullptr,
                                            (double*)dmdt_out, p->alpha, true, nullptr);
    if (e != hipSuccess) return hip_fail(e, "mm_llg_rhs");
    return MM_OK;
}

mm_status mm_llg_step(mm_plan* pl, void* m, const double h_ext[3], unsigned terms, double* t,
                      double* dt, const mm_step_opts* o, mm_step_stats* st)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !t || !dt || !o) {
        set_error("null argument");
        return MM_EINVAL;
    }
    if (!(o->rtol > 0.0) || !(o->atol > 0.0) || o->max_steps < 0 ||
        (o->method != MM_DP45 && o->method != MM_RKF45)) {
        set_error("rtol and atol must be positive, max_steps non-negative, method DP45 or RKF45");
        return MM_EINVAL;
    }
    const double dt_min = o->dt_min > 0.0 ? o->dt_min : 1e-20;
    return p->prec == MM_FP32
               ? dp45<float>(p, m, h_ext, terms, t, dt, o->rtol, o->atol, o->t_end, o->max_steps,
                             dt_min, o->renorm != 0, false, 0.0, st, o->method)
               : dp45<double>(p, m, h_ext, terms, t, dt, o->rtol, o->atol, o->t_end, o->max_steps,
                              dt_min, o->renorm != 0, false, 0.0, st, o->method);
}

// FP32 relaxation with a double state: the device-controlled steps of the
// request server on this plan (the state and trial state in double, stage
// inputs rounded once to float with their residual in the exchange
// differences).  With a float state the rounding noise, amplified by the
// stiffest exchange modes at the step size the controller settles on, holds
// the torque of some relaxations near 1e-5.  The host polls the controller
// every 16 steps; steps after completion change nothing.
static mm_status relax_split(Plan* p, void* m, const double h_ext[3], unsigned terms, double tol,
                             long max_steps, double rtol, mm_step_stats* st)
{
    const bool was = p->state64;
    p->state64 = true;
    mm_status s = ensure_rk(p);
    DevCtl c{};
    if (s == MM_OK) {
        c.t = 0.0;
        c.dt = -1.0;
        c.t_end = std::numeric_limits<double>::infinity();
        c.dt_min = 1e-20;
        c.torque_tol = tol;
        c.max_steps = max_steps;
        c.relax = 1;
        c.renorm = 1;
        s = dev_prepare<float>(p, m, h_ext, terms, c, rtol, rtol);
    }
    while (s == MM_OK) {
        for (int i = 0; i < 16 && s == MM_OK; ++i)
            s = dev_step<float>(p, h_ext, terms, rtol, rtol, true, true);
        if (s != MM_OK) break;
        hipError_t e = hipMemcpyAsync(&c, p->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) s = hip_fail(e, "reading the step controller");
        if (s == MM_OK && c.done) break;
    }
    if (s == MM_OK) {
        hipError_t e = dev_result(p, m);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) s = hip_fail(e, "copying the result");
    }
    p->state64 = was;
    if (s != MM_OK) return s;
    if (st) {
        st->accepted = c.accepted;
        st->rejected = c.rejected;
        st->rhs_evals = c.rhs_evals;
        st->t = c.t;
        st->dt = c.dt;
        st->err_last = c.err_last;
    }
    if (c.result == MM_ENOTCONV) set_error("relaxation did not reach the torque criterion");
    if (c.result == MM_EDTMIN) set_error("step size fell below dt_min");
    if (c.result == MM_ENONFINITE) set_error("non-finite magnetisation");
    return (mm_status)c.result;
}

mm_status mm_relax(mm_plan* pl, void* m, const double h_ext[3], unsigned terms, double tol,
                   long max_steps, double rtol, mm_step_stats* st)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m) {
        set_error("null argument");
        return MM_EINVAL;
    }
    if (!(tol > 0.0) || !(rtol > 0.0) || max_steps < 0) {
        set_error("tol and rtol must be positive, max_steps non-negative");
        return MM_EINVAL;
    }
    double t = 0.0, dt = -1.0;
    const double inf = std::numeric_limits<double>::infinity();
    if (split_state_ok(*p, terms)) return relax_split(p, m, h_ext, terms, tol, max_steps, rtol, st);
    return p->prec == MM_FP32
               ? dp45<float>(p, m, h_ext, terms, &t, &dt, rtol, rtol, inf, max_steps, 1e-20, true,
                             true, tol, st)
               : dp45<double>(p, m, h_ext, terms, &t, &dt, rtol, rtol, inf, max_steps, 1e-20, true,
                              true, tol, st);
}

mm_status mm_energy(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms, double t,
                    double E[6])
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !E) {
        set_error("null argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32 ? energy_impl<float>(p, (const float*)m, h_ext, terms, t, E)
                              : energy_impl<double>(p, (const double*)m, h_ext, terms, t, E);
}

mm_status mm_energy_noalloc(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms,
                            double t, double E[6])
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !E) {
        set_error("null argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32 ? energy_noalloc_impl<float>(p, (const float*)m, h_ext, terms, t, E)
                              : energy_noalloc_impl<double>(p, (const double*)m, h_ext, terms, t, E);
}

mm_status mm_max_torque(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms,
                        double t, double* out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !out) {
        set_error("null argument");
        return MM_EINVAL;
    }
    hipError_t e = p->prec == MM_FP32
                       ? eval_field<float>(*p, (const float*)m, h_ext, terms, t, nullptr, nullptr,
                                           p->alpha, true, p->red_out + 1)
                       : eval_field<double>(*p, (const double*)m, h_ext, terms, t, nullptr,
                                            nullptr, p->alpha, true, p->red_out + 1);
    if (e != hipSuccess) return hip_fail(e, "mm_max_torque");
    mm_status s = fetch(p, 2);
    if (s != MM_OK) return s;
    *out = p->host_out[1];
    return MM_OK;
}

mm_status mm_heff_vjp(mm_plan* pl, const void* m, const void* w, unsigned terms, void* grad_m,
                      void* grad_ms)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !w || !grad_m || grad_m == m || grad_m == w) {
        set_error("null or aliased argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32
               ? heff_vjp_impl<float>(p, (const float*)m, (const float*)w, nullptr, terms, 0.0, false,
                                      (float*)grad_m, (float*)grad_ms)
               : heff_vjp_impl<double>(p, (const double*)m, (const double*)w, nullptr, terms, 0.0,
                                       false, (double*)grad_m, (double*)grad_ms);
}

mm_status mm_llg_rhs_vjp(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms,
                         double t, const void* w, void* grad_m, void* grad_ms)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !w || !grad_m || grad_m == m || grad_m == w) {
        set_error("null or aliased argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32
               ? heff_vjp_impl<float>(p, (const float*)m, (const float*)w, h_ext, terms, t, true,
                                      (float*)grad_m, (float*)grad_ms)
               : heff_vjp_impl<double>(p, (const double*)m, (const double*)w, h_ext, terms, t, true,
                                       (double*)grad_m, (double*)grad_ms);
}

mm_status mm_rk4_forward(mm_plan* pl, void* m, const double h_ext[3], unsigned terms, double t0,
                         double dt, long nsteps, const unsigned char* region, long ckpt_every,
                         void* ckpt, double* loss)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || nsteps < 0 || !(dt > 0.0) || (ckpt && ckpt_every <= 0)) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32 ? rk4_forward_impl<float>(p, m, h_ext, terms, t0, dt, nsteps, region,
                                                        ckpt_every, ckpt, loss)
                              : rk4_forward_impl<double>(p, m, h_ext, terms, t0, dt, nsteps, region,
                                                         ckpt_every, ckpt, loss);
}

mm_status mm_rk4_adjoint(mm_plan* pl, const void* ckpt, const double h_ext[3], unsigned terms,
                         double t0, double dt, long nsteps, const unsigned char* region,
                         long ckpt_every, void* grad_ms, void* grad_m0, double* loss)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (p && nonlinear_anis(p, terms)) {
        set_error("higher-order anisotropy is not linear in m: no adjoint");
        return MM_EINVAL;
    }
    if (p && (stencil_extended(p, terms) || p->layered)) {
        set_error("per-cell exchange, per-cell Ku, DMI and thin layers have no adjoint");
        return MM_EINVAL;
    }
    if (!p || !ckpt || !region || nsteps <= 0 || !(dt > 0.0) || ckpt_every <= 0) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32 ? rk4_adjoint_impl<float>(p, ckpt, h_ext, terms, t0, dt, nsteps, region,
                                                        ckpt_every, grad_ms, grad_m0, loss)
                              : rk4_adjoint_impl<double>(p, ckpt, h_ext, terms, t0, dt, nsteps,
                                                         region, ckpt_every, grad_ms, grad_m0, loss);
}

mm_status mm_profile(mm_plan* pl, int enable)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p) {
        set_error("null plan");
        return MM_EINVAL;
    }
    hipError_t e = prof_flush(*p);
    if (e != hipSuccess) return hip_fail(e, "mm_profile");
    if (enable) {
        for (int i = 0; i < MM_NPASS; ++i) {
            p->prof.ms[i] = 0.0;
            p->prof.cnt[i] = 0;
        }
    }
    p->prof.on = enable != 0;
    return MM_OK;
}

mm_status mm_profile_read(mm_plan* pl, double ms[], long count[])
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !ms || !count) {
        set_error("null argument");
        return MM_EINVAL;
    }
    hipError_t e = prof_flush(*p);
    if (e != hipSuccess) return hip_fail(e, "mm_profile_read");
    for (int i = 0; i < MM_NPASS; ++i) {
        ms[i] = p->prof.ms[i];
        count[i] = p->prof.cnt[i];
    }
    return MM_OK;
}

mm_status mm_debug_kernel(mm_plan* pl, int s, void* out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !out || s < 0 || s > 5 || p->layered) {
        set_error("invalid argument (not available for thin layers)");
        return MM_EINVAL;
    }
    hipError_t e = debug_kernel(*p, s, (double*)out);
    if (e != hipSuccess) return hip_fail(e, "mm_debug_kernel");
    return MM_OK;
}

mm_status mm_debug_spectrum(mm_plan* pl, int s, void* out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !out || s < 0 || s > 5 || p->layered) {
        set_error("invalid argument (not available for thin layers)");
        return MM_EINVAL;
    }
    hipError_t e = p->prec == MM_FP32 ? debug_spectrum<float>(*p, s, (double*)out)
                                      : debug_spectrum<double>(*p, s, (double*)out);
    if (e != hipSuccess) return hip_fail(e, "mm_debug_spectrum");
    return MM_OK;
}

}  // extern "C"
