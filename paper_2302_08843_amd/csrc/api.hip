// api.hip -- the C ABI declared in include/mm.h: plan life cycle, argument
// checks, and the host-side step-size controller of the Dormand-Prince
// integrator (the device computes the stages, the error norm and the torque;
// the host receives 8 bytes per step and decides).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>

#include "engine.h"

namespace mmx {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

static int padded_extent(int n)
{
    if (n <= 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return p;
}

static size_t elem_size(const Plan& p) { return p.prec == MM_FP32 ? 4 : 8; }

static mm_status hip_fail(hipError_t e, const char* what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EHIP;
}

#define MM_HIP(call, what)                               \
    do {                                                 \
        hipError_t e__ = (call);                         \
        if (e__ != hipSuccess) return hip_fail(e__, what); \
    } while (0)

static void free_plan(Plan* p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    for (auto& r : p->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : p->prof.pool) (void)hipEventDestroy(e);
    void* bufs[] = {p->Khat, p->S1, p->S2 == p->S1 ? nullptr : p->S2, p->tw, p->Ms_cell,
                    p->mask, p->rk, p->red, p->red_out};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->host_out) (void)hipHostFree(p->host_out);
    delete p;
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

static mm_status ensure_rk(Plan* p)
{
    if (p->rk) return MM_OK;
    return alloc(p, &p->rk, 10 * 3 * (size_t)p->N * elem_size(*p), "Runge-Kutta buffers");
}

template <typename T>
static T* rk_vec(Plan* p, int i)
{
    return (T*)p->rk + (size_t)i * 3 * p->N;
}

static mm_status fetch(Plan* p, int n)
{
    MM_HIP(hipMemcpyAsync(p->host_out, p->red_out, sizeof(double) * n, hipMemcpyDeviceToHost,
                          p->stream),
           "reading a reduction");
    MM_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
    return MM_OK;
}

// ---------------------------------------------------------------------------
// Dormand-Prince driver.  mode_relax: alpha = 1, no precession, renormalise,
// stop on the torque criterion.
// ---------------------------------------------------------------------------
template <typename T>
static mm_status dp45(Plan* p, void* m_user, const double hext[3], unsigned terms, double* t,
                      double* dt, double rtol, double atol, double t_end, long max_steps,
                      double dt_min, bool renorm, bool relax, double torque_tol,
                      mm_step_stats* st)
{
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
        // Hairer-Norsett-Wanner starting step
        MM_HIP(start_norms<T>(*p, y, k[0], nullptr, rtol, atol, p->red_out + 2), "start norms");
        s = fetch(p, 5);
        if (s != MM_OK) return s;
        const double cnt = 3.0 * (double)p->n_magnetic;
        const double d0 = cnt > 0 ? std::sqrt(p->host_out[2] / cnt) : 0.0;
        const double d1 = cnt > 0 ? std::sqrt(p->host_out[3] / cnt) : 0.0;
        const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
        const double one = 1.0;
        T* f0 = k[0];
        MM_HIP(rk_combine<T>(*p, ys, y, h0, &one, &f0, 1), "start step");
        MM_HIP(eval_field<T>(*p, ys, hext, terms, *t + h0, nullptr, k[1], alpha, precess, nullptr),
               "right-hand side");
        loc.rhs_evals++;
        MM_HIP(start_norms<T>(*p, y, k[0], k[1], rtol, atol, p->red_out + 2), "start norms");
        s = fetch(p, 5);
        if (s != MM_OK) return s;
        const double d2 = (cnt > 0 ? std::sqrt(p->host_out[4] / cnt) : 0.0) / h0;
        const double mx = std::max(d1, d2);
        const double h1 = mx <= 1e-15 ? std::max(1e-6, h0 * 1e-3) : std::pow(0.01 / mx, 0.2);
        *dt = std::min(100.0 * h0, h1);
    }
    double E[7];
    for (int j = 0; j < 7; ++j) E[j] = kB5[j] - kB4[j];
    bool last_rejected = false;
    double torque = std::numeric_limits<double>::infinity();
    bool torque_known = false;
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
        for (int sg = 1; sg < 7; ++sg) {
            T* target = sg == 6 ? y1 : ys;
            MM_HIP(rk_combine<T>(*p, target, y, h, kA[sg], k, sg), "stage input");
            MM_HIP(eval_field<T>(*p, target, hext, terms, *t + kC[sg] * h, nullptr, k[sg], alpha,
                                 precess, nullptr),
                   "right-hand side");
            loc.rhs_evals++;
        }
        MM_HIP(rk_error_norm<T>(*p, y, y1, h, E, k, 7, rtol, atol, p->red_out), "error norm");
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
            if (renorm) {
                MM_HIP(renormalise<T>(*p, y), "renormalise");
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

}  // namespace mmx

using namespace mmx;

namespace mmx {

template <typename T>
static mm_status energy_impl(Plan* p, const T* m, const double h_ext[3], unsigned terms, double t,
                             double E[5])
{
    mm_status s = ensure_rk(p);
    if (s != MM_OK) return s;
    T* h = rk_vec<T>(p, 0);
    const unsigned bits[4] = {MM_DEMAG, MM_EXCH, MM_ANIS, MM_ZEEMAN};
    for (int e = 0; e < 4; ++e) {
        if (!(terms & bits[e])) {
            MM_HIP(hipMemsetAsync(p->red_out + e, 0, sizeof(double), p->stream), "clear");
            continue;
        }
        MM_HIP(eval_field<T>(*p, m, h_ext, bits[e], t, h, nullptr, p->alpha, true, nullptr),
               "field");
        MM_HIP(dot_ms<T>(*p, m, h, p->red_out + e), "energy reduction");
    }
    s = fetch(p, 4);
    if (s != MM_OK) return s;
    const double V = p->d[0] * p->d[1] * p->d[2];
    double tot = 0.0;
    for (int e = 0; e < 4; ++e) {
        E[e] = (e == 3 ? -1.0 : -0.5) * kMu0 * V * p->host_out[e];
        tot += E[e];
    }
    E[4] = tot;
    return MM_OK;
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
    Plan* p = new Plan();
    for (int a = 0; a < 3; ++a) {
        p->n[a] = grid[a];
        p->d[a] = cell[a];
        p->P[a] = padded_extent(grid[a]);
        p->eu[a] = o.ku_axis[a] / nrm;
    }
    p->N = (long)grid[0] * grid[1] * grid[2];
    p->Hx = p->P[0] > 1 ? p->P[0] / 2 + 1 : 1;
    // spectral rows start on 128-byte boundaries for the real kernel array
    // (32 floats or 16 doubles) and therefore for the complex spectra too
    const int row_align = o.prec == MM_FP32 ? 32 : 16;
    p->Hxp = (p->Hx + row_align - 1) / row_align * row_align;
    p->S1n = 3L * grid[2] * grid[1] * p->Hxp;
    p->S2n = 3L * grid[2] * p->P[1] * p->Hxp;
    p->Kn = (long)(p->P[2] / 2 + 1) * (p->P[1] / 2 + 1) * p->Hxp;
    p->Lmax = std::max(p->P[0], std::max(p->P[1], p->P[2]));
    p->prec = o.prec;
    p->Ms = Ms;
    p->A = A;
    p->Ku = Ku;
    p->alpha = alpha;
    p->demag_p = o.demag_p;
    p->percell = false;
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
#define MM_ALLOC(ptr, bytes, what)                              \
    do {                                                        \
        s = alloc(p, (void**)&(ptr), (bytes), what);            \
        if (s != MM_OK) {                                       \
            free_plan(p);                                       \
            return s;                                           \
        }                                                       \
    } while (0)
    MM_ALLOC(p->Khat, 6 * (size_t)p->Kn * es, "spectral kernel");
    MM_ALLOC(p->S1, (size_t)p->S1n * 2 * es, "spectrum S1");
    if (p->P[2] > 1 && p->P[1] > 1)
        MM_ALLOC(p->S2, (size_t)p->S2n * 2 * es, "spectrum S2");
    else
        p->S2 = p->S1;
    MM_ALLOC(p->tw, (size_t)p->Lmax * 2 * es, "twiddles");
    MM_ALLOC(p->red, sizeof(double) * kRedSlots, "reduction partials");
    MM_ALLOC(p->red_out, sizeof(double) * 8, "reduction results");
#undef MM_ALLOC
    hipError_t e = hipHostMalloc((void**)&p->host_out, sizeof(double) * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "pinned host buffer");
    }
    e = p->prec == MM_FP32 ? init_twiddles<float>(*p) : init_twiddles<double>(*p);
    if (e == hipSuccess) e = p->prec == MM_FP32 ? build_tensor<float>(*p) : build_tensor<double>(*p);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        mm_status st = hip_fail(e, "building the demag kernel");
        free_plan(p);
        return st;
    }
    *out = reinterpret_cast<mm_plan*>(p);
    return MM_OK;
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
    if (!(o->rtol > 0.0) || !(o->atol > 0.0) || o->max_steps < 0) {
        set_error("rtol and atol must be positive, max_steps non-negative");
        return MM_EINVAL;
    }
    const double dt_min = o->dt_min > 0.0 ? o->dt_min : 1e-20;
    return p->prec == MM_FP32
               ? dp45<float>(p, m, h_ext, terms, t, dt, o->rtol, o->atol, o->t_end, o->max_steps,
                             dt_min, o->renorm != 0, false, 0.0, st)
               : dp45<double>(p, m, h_ext, terms, t, dt, o->rtol, o->atol, o->t_end, o->max_steps,
                              dt_min, o->renorm != 0, false, 0.0, st);
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
    return p->prec == MM_FP32
               ? dp45<float>(p, m, h_ext, terms, &t, &dt, rtol, rtol, inf, max_steps, 1e-20, true,
                             true, tol, st)
               : dp45<double>(p, m, h_ext, terms, &t, &dt, rtol, rtol, inf, max_steps, 1e-20, true,
                              true, tol, st);
}

mm_status mm_energy(mm_plan* pl, const void* m, const double h_ext[3], unsigned terms, double t,
                    double E[5])
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !m || !E) {
        set_error("null argument");
        return MM_EINVAL;
    }
    return p->prec == MM_FP32 ? energy_impl<float>(p, (const float*)m, h_ext, terms, t, E)
                              : energy_impl<double>(p, (const double*)m, h_ext, terms, t, E);
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
    if (!p || !out || s < 0 || s > 5) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    hipError_t e = debug_kernel(*p, s, (double*)out);
    if (e != hipSuccess) return hip_fail(e, "mm_debug_kernel");
    return MM_OK;
}

mm_status mm_debug_spectrum(mm_plan* pl, int s, void* out)
{
    Plan* p = reinterpret_cast<Plan*>(pl);
    if (!p || !out || s < 0 || s > 5) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    hipError_t e = p->prec == MM_FP32 ? debug_spectrum<float>(*p, s, (double*)out)
                                      : debug_spectrum<double>(*p, s, (double*)out);
    if (e != hipSuccess) return hip_fail(e, "mm_debug_spectrum");
    return MM_OK;
}

}  // extern "C"
