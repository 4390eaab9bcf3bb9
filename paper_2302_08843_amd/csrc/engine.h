// engine.h -- internal plan state and the device-side pipeline of the
// micromagnetic hot path (not part of the public ABI, see include/mm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/mm.h"

namespace mmx {

// Physical constants: mu0 = 4 pi 1e-7 (the paper does not print it) and the
// reduced gyromagnetic ratio printed with the LLG equation (Sec. 3).
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kGamma = 2.21e5;

// Largest padded FFT length per axis handled by the kernels.
constexpr int kMaxFFT = 1024;
constexpr int kMaxLayers = 16;  // thin layers of unequal height per plan

constexpr int kRedSlots = 8192;

// Event-based per-pass timing (mm_profile).
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Rec {
        int pass;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    double ms[MM_NPASS] = {};
    long cnt[MM_NPASS] = {};
};

struct DevCtl;
// A spectral kernel and twiddle table shared by plans of one grid class
// (same grid, precision, near-field order and cell proportions: the demag
// tensor depends only on the cell shape, not its size).  Freed with its last
// owner.
struct SharedTensor {
    void *Khat = nullptr, *tw = nullptr;
    size_t bytes = 0;
    int refs = 0;
};

struct Plan {
    // geometry
    int n[3];      // nx, ny, nz
    double d[3];   // dx, dy, dz
    int P[3];      // padded extents
    int Hx;        // Px/2 + 1 (1 when Px == 1): x bins kept by the real transform
    int Hxp;       // row stride of every spectral array (Hx rounded up to 128 bytes of reals)
    long N;        // cells
    long S1n;      // complex values in S1 = 3 * nz * ny * Hxp
    long S2n;      // complex values in S2 = 3 * nz * Py * Hxp
    long Kn;       // reals per spectral-tensor component (Pz/2+1)(Py/2+1) Hxp
    int Lmax;      // twiddle table length = max(P)
    // material
    int prec;      // MM_FP32 / MM_FP64
    double Ms, A, Ku, alpha;
    double eu[3];
    double Ku2, Kc1, Kc2;  // higher-order anisotropy
    double ec[3][3];       // cubic principal axes (orthonormal rows)
    int demag_p;
    bool percell;  // per-cell Ms present
    bool percell_A;  // per-cell exchange constant present (A_cell)
    bool percell_Ku = false;  // per-cell first-order uniaxial constant present (Ku_cell)
    bool dmi;        // DMI term present
    int dmi_type;    // MM_DMI_INTERFACE / _BULK / _D2D
    double D;        // uniform DMI strength (ignored with D_cell)
    bool percell_D;  // per-cell DMI strength present (D_cell)
    bool dmi_mixed;  // D_cell holds strengths of both signs
    // thin layers of unequal height (Sec. 4.4): nz > 1 layers, no z padding;
    // the demag spectrum is coupled densely across layers per (kx, ky)
    bool layered = false;
    std::vector<double> zb;  // layer bottoms, nz + 1 values (zb[0] = 0)
    double edmi[3][3];  // DMI vectors e^dmi_x, e^dmi_y, e^dmi_z
    long n_magnetic;  // magnetic cells (Ms > 0)
    // drive
    bool drive;
    double drive_amp[3], drive_freq;
    hipStream_t stream;
    int ncu = 256;  // compute units of the device (persistent launches)
    // device buffers (element type = plan precision unless noted)
    void *Khat = nullptr;     // [6][Pz/2+1][Py/2+1][Hxp] real, scaled by 1/(Px Py Pz)
    void *S1 = nullptr;       // [3][nz][ny][Hxp] complex
    void *S2 = nullptr;       // [3][nz][Py][Hxp] complex (aliases S1 when Py == 1)
    void *tw = nullptr;       // Lmax complex roots exp(-2 pi i n / Lmax)
    void *Ms_cell = nullptr;  // N reals, or null
    void *A_cell = nullptr;   // N reals (per-cell exchange constant), or null
    void *Ku_cell = nullptr;  // N reals (per-cell uniaxial constant), or null
    void *D_cell = nullptr;   // N reals (per-cell DMI strength), or null
    void *zw = nullptr;       // layered: 4 reals per layer (z exchange down/up, 1/(2 dz_k), 0)
    double *lw = nullptr;     // layered: nz doubles, the layer heights (energy weights)
    // Oersted field (allocated on first use)
    void *oe_G = nullptr;     // [3][Pz/2+1][Py/2+1][Hxp] real: Im of the kernel spectrum / (Px Py Pz)
    void *h_oe = nullptr;     // 3N reals: field of the set current density
    bool oe_on = false;       // Oersted term present (mm_set_current)
    double oe_freq = 0.0;     // h_oe scaled by sin(2 pi f t) when f != 0
    unsigned char *mask = nullptr;  // N bytes drive mask, or null
    // Runge-Kutta work space (allocated on first use)
    void *rk = nullptr;       // 10 vectors of 3N
    double *red = nullptr;    // reduction partials (kRedSlots doubles)
    double *red_out = nullptr;  // reduction results (8 doubles)
    double *host_out = nullptr; // pinned host mirror of red_out
    // differentiation work space (allocated on first use)
    void *adj = nullptr;        // 16 vectors of 3N
    void *seg = nullptr;        // stage states and fields of one checkpoint segment
    size_t seg_bytes = 0;
    double *gms = nullptr;      // N doubles: Ms-gradient accumulator
    DevCtl *ctl = nullptr;      // device-side step controller
    SharedTensor *shared = nullptr;  // Khat and tw owned jointly with other plans
    bool ws = false;  // Khat, S1, S2, tw, red, red_out, rk, ctl carved from a caller workspace
    // FP32 plans, device-controlled runs: Runge-Kutta state in double (6N
    // doubles: y, then the trial state y1), stages in float
    bool state64 = false;
    double *st64 = nullptr;
    // A batch of requests of one grid (request server): S1, S2, the
    // Runge-Kutta vectors and st64 hold `batch` requests each, request b
    // after b - 1 (vector v of request b at v * vstride + b * 3N); ctl, the
    // reduction slots (8 doubles per request in red_out) likewise.  Pb: one
    // LocalParams per request (device), Ms_b: one Ms per request (device, in
    // the plan's precision).  vstride: elements between Runge-Kutta vectors
    // (0: 3N; a view of one request of a batch keeps the batch's stride).
    double *epart = nullptr;  // error-norm partials of the local pass, 2 ny nz doubles
    int batch = 1;
    long vstride = 0;
    void *Pb = nullptr;
    void *Ms_b = nullptr;
    void *Pb_host = nullptr;  // pinned staging of Pb and Ms_b, one entry per request
    size_t bytes = 0;
    Profiler prof;
};

// Record an event pair around one launch when profiling is on.
hipError_t prof_begin(Plan &p, int pass, hipEvent_t *a);
hipError_t prof_end(Plan &p, int pass, hipEvent_t a);
hipError_t prof_flush(Plan &p);

// Thread-local error message (mm_last_error).
void set_error(const std::string &msg);

// Device pipeline, instantiated for float and double in kernels.hip.
template <typename T>
hipError_t build_tensor(Plan &p);
template <typename T>
hipError_t init_twiddles(Plan &p);

// Field / right-hand side evaluation at state m (3N) and time t.
//   h_out    : effective field (may be null)
//   dm_out   : LLG right-hand side (may be null), with alpha_eff and precess
//   torque   : if non-null, per-block maxima of |m x h|/Ms into p.red and the
//              final maximum into *torque (device double)
//   m_lo     : if non-null (FP32, plain stencil), the state is m + m_lo, the
//              float rounding residual of a double state, and the exchange
//              differences take it into account
template <typename T>
hipError_t eval_field(Plan &p, const T *m, const double hext[3], unsigned terms, double t,
                      T *h_out, T *dm_out, double alpha_eff, bool precess, double *torque,
                      const T *m_lo = nullptr);

// A Runge-Kutta stage input ys = y + sum_{j < nk} c_j k_j (c_j multiplied by
// *h when h is not null), formed by the x forward pass as it loads its rows.
template <typename T>
struct StageIn {
    const T *y = nullptr;
    const T *k[7] = {};
    double c[7] = {};
    const double *h = nullptr;
    T *ys = nullptr;
    int nk = 0;
    // optional: the partial error sum_{j < nk} e_j k_j (e_j multiplied by *h
    // like c_j), formed in double from the same loads and stored to ep
    T *ep = nullptr;
    double e[7] = {};
};

// The Dormand-Prince error norm accumulated by the local pass of the last
// stage: per component e = ep + e6 k6 (ep from the x forward pass, k6 the
// right-hand side just computed), sc = atol + rtol max(|y|, |y1|) with y1 the
// stage input; out_dev[0] = RMS of e / sc over magnetic components,
// out_dev[5] = number of non-finite entries of y.
template <typename T>
struct ErrIn {
    const T *y = nullptr;
    double e6 = 0.0;
    double rtol = 0.0, atol = 0.0;
    double *out_dev = nullptr;
};
// Right-hand side at a stage input: ys (3N, 16-byte aligned like y and the
// k_j) is written by the x forward pass, which forms it on the fly, and the
// local pass reads it; without the demag term, or on grids whose x extent
// is 1, the combination runs as a kernel of its own first.  The arithmetic
// of ys is that of rk_combine.
template <typename T>
hipError_t eval_field_stage(Plan &p, const StageIn<T> &sc, const double hext[3], unsigned terms,
                            double t, T *dm_out, double alpha_eff, bool precess, double *torque,
                            const ErrIn<T> *err = nullptr);
// Whether eval_field_stage can accumulate the error norm (ErrIn, sc.ep set)
// for this plan and terms: the demag chain runs, the plain stencil, one
// request, the wave-local local pass, the partials buffer in place.
bool err_fusable(const Plan &p, unsigned terms);
// whether device-controlled steps with a double state and the split-state
// exchange can run on this plan and terms: FP32, one request, uniform Ms,
// plain stencil, equal layers, static fields
bool split_state_ok(const Plan &p, unsigned terms);

// y_out = y + h * sum_j a[j] k[j]  (nk <= 7).  hdev: if not null, h is read
// from this device double instead (device-side step control).
template <typename T>
hipError_t rk_combine(Plan &p, T *y_out, const T *y, double h, const double *a, T *const *k,
                      int nk, const double *hdev = nullptr);
// RMS error norm of e = h sum_j e[j] k[j] scaled by atol + rtol max(|y|,|y1|)
// over magnetic components into out_dev[0]; the number of non-finite entries
// of y into out_dev[5].  ctl (device-controlled steps): the same launch then
// takes the step's accept / reject decision and next step size on out_dev.
template <typename T>
hipError_t rk_error_norm(Plan &p, const T *y, const T *y1, double h, const double *e,
                         T *const *k, int nk, double rtol, double atol, double *out_dev,
                         const double *hdev = nullptr, DevCtl *ctl = nullptr);

// Device-side Dormand-Prince controller state (one per plan in device
// memory).  Every decision the host-driven loop takes from a synchronised
// read-back is taken here by single-thread kernels, so a sequence of steps can
// be enqueued (or captured in a HIP graph) without a host round trip.
struct DevCtl {
    double t, dt, h, t_end, dt_min, torque_tol, torque, err_last;
    long accepted, rejected, rhs_evals, max_steps;
    int done;      // 0 while stepping, 1 once finished (then every step is a no-op)
    int result;    // mm_status of a finished run
    int last_rejected, commit, relax, renorm;
};
// start of a step: a relaxation takes its torque from p.red_out[1] (left
// there by the previous step's closing evaluation, or dp_torque at the
// start); finish on the torque criterion / step cap / t_end, else set the
// trial step h = min(dt, t_end - t)
hipError_t dp_begin(Plan &p, DevCtl *c);
// (accept / reject and the new step size: in the error norm's final launch,
// rk_error_norm / rk_error_norm_d with ctl)
// on acceptance: y = y1 (renormalised if c->renorm) and, without renorm,
// k0 = k6 (first-same-as-last)
template <typename T>
hipError_t dp_commit(Plan &p, DevCtl *c, T *y, const T *y1, T *k0, const T *k6);
// Double state with FP32 stages (Plan::state64): stage inputs formed in
// double from y and rounded to float into ys (and kept in double in y1 when
// not null; with ys_lo, the rounding residual float(v - ys) too); the error
// norm from double y, y1; the commit in double, which with renormalisation
// leaves the rounded state in ys (and its residual in ys_lo) -- the
// renormalised y1 on acceptance, the unchanged y on rejection; conversions.
hipError_t rk_combine_d(Plan &p, float *ys, double *y1, const double *y, const double *a,
                        float *const *k, int nk, const double *hdev, float *ys_lo = nullptr);
hipError_t rk_error_norm_d(Plan &p, const double *y, const double *y1, const double *e,
                           float *const *k, int nk, double rtol, double atol, double *out_dev,
                           const double *hdev, DevCtl *ctl = nullptr);
hipError_t dp_commit_d(Plan &p, DevCtl *c, double *y, const double *y1, float *ys, float *k0,
                       const float *k6, float *ys_lo = nullptr);
hipError_t convert_f32_f64(Plan &p, const float *in, double *out, long n);
hipError_t convert_f64_f32(Plan &p, const double *in, float *out, long n);
// c->torque = p.red_out[1] while running
hipError_t dp_torque(Plan &p, DevCtl *c);
// Renormalise |m| = 1 on magnetic cells, zero m on vacuum cells.
template <typename T>
hipError_t renormalise(Plan &p, T *m);
// anisotropy energy density (all orders) summed over magnetic cells -> *out_dev
// (block partials in `partials`, kRedSlots doubles, or the plan's red)
template <typename T>
hipError_t anis_energy(Plan &p, const T *m, double *out_dev, double *partials = nullptr);
// sum over cells of Ms * (a . b) in double -> *out_dev (partials as above)
template <typename T>
hipError_t dot_ms(Plan &p, const T *a, const T *b, double *out_dev, double *partials = nullptr);
// Hairer-Norsett-Wanner starting-step norms: sums of (y/sc)^2, (f/sc)^2 and
// ((f1 - f0)/sc)^2 with sc = atol + rtol |y|, into out_dev[0..2]
template <typename T>
hipError_t start_norms(Plan &p, const T *y, const T *f0, const T *f1, double rtol, double atol,
                       double *out_dev);
// Count magnetic cells (Ms > 0) into *out_dev.
template <typename T>
hipError_t count_magnetic(Plan &p, double *out_dev);
// Oersted field h_out (3N) of the current density j (3N), both of the plan's
// precision: FFT convolution with the cell-averaged Biot-Savart kernel, through
// the demag passes with the cross product in the last-axis pass.  The kernel
// spectrum is built and kept on first use.
template <typename T>
hipError_t oersted_field(Plan &p, const T *j, T *h_out);
// Numbers of negative and positive entries of v (N values) into out_dev[0..1].
template <typename T>
hipError_t count_signs(Plan &p, const T *v, double *out_dev);
// Transposed field / LLG right-hand side.  With h == nullptr: nu = H^T w
// (w masked to magnetic cells).  With h (the field at m): nu = J^T w of the
// LLG right-hand side with damping alpha.  gms (double, may be null)
// accumulates d(w.h)/dMs resp. d(w.f)/dMs.  g_tmp and z_tmp are 3N scratch.
template <typename T>
hipError_t field_vjp(Plan &p, const T *m, const T *w, const T *h, unsigned terms, double alpha,
                     T *g_tmp, T *z_tmp, T *nu, double *gms);
// out = sum_{j < nk} c[j] v[j]  (nk <= 6)
template <typename T>
hipError_t lincomb(Plan &p, T *out, const double *c, T *const *v, int nk);
// *out_dev += scale * sum over region of m_z
template <typename T>
hipError_t region_mz_accum(Plan &p, const T *m, const unsigned char *region, double *out_dev,
                           double scale);
// lam_z += val on the region
template <typename T>
hipError_t add_region(Plan &p, T *lam, const unsigned char *region, double val);
hipError_t zero_doubles(Plan &p, double *ptr, long n);
template <typename T>
hipError_t from_double(Plan &p, const double *in, T *out, long n);
// Debug: real-space kernel (component s) placed in the padded grid, doubles.
// ---- Host-side plan services (api.hip), also used by the request server ----
void set_error(const std::string &msg);
mm_status hip_fail(hipError_t e, const char *what);
void free_plan(Plan *p);
void release_tensor(SharedTensor *t);
mm_status ensure_rk(Plan *p);
mm_status plan_build(const int grid[3], const double cell[3], double Ms, double A, double Ku,
                     double alpha, const mm_opts &o, SharedTensor *share, Plan **out,
                     int batch = 1);
// Device bytes of a batch plan of `batch` requests of this grid for the
// request server (no spectral kernel), with the double state when state64.
size_t batch_footprint(const int grid[3], int prec, int batch, bool state64);
// Request b of a batch plan as a plan of its own (views into the batch's
// buffers; never freed, owns nothing).
Plan batch_view(const Plan &g, int b);
// Slot b of a batch plan takes the constants of request view v (material,
// cell, field h_ext, terms, alpha_eff / precession): staged in pinned memory
// and copied on g's stream.  Uniform material and the plain stencil only.
hipError_t batch_set_slot(Plan &g, int b, const Plan &v, const double hext[3], unsigned terms,
                          double alpha_eff, bool precess);
// Bytes of one request's constants in a batch plan (Pb entry + Ms entry).
size_t batch_slot_bytes();
// Every slot of a batch plan empty: the plan's geometry with no material
// (zero field and right-hand side), Ms 0; on g's stream from its staging.
hipError_t batch_init_slots(Plan &g);
// Zero-padded FFT extent along an axis of n cells: 1 for n = 1, else the
// smallest power of two >= 2n - 1.
int padded_extent(int n);
// Whether requests of this grid can share launches (the batched kernels
// cover its transform lengths: x extent at least 2).
bool batch_supported(const int grid[3], int prec);
size_t plan_footprint(const int grid[3], int prec, bool with_tensor);
// Byte offsets of a plan's persistent buffers inside one workspace, each
// aligned to 256 bytes (equal layers): spectral kernel, spectra, twiddles,
// reduction buffers, Runge-Kutta vectors and the step controller.
struct WsLayout {
    size_t Khat, S1, S2, tw, red, red_out, rk, ctl, epart, total;
    bool s2_separate;
};
WsLayout ws_layout(const int grid[3], int prec);
// Device-controlled Dormand-Prince run: dev_prepare copies m0 into the
// state, evaluates f(y0) (and the torque for relaxation), picks the starting
// step if init.dt <= 0, uploads the controller (synchronises); dev_step
// enqueues one step without synchronising; dev_state is the state buffer.
template <typename T>
mm_status dev_prepare(Plan *p, const void *m0, const double hext[3], unsigned terms,
                      const DevCtl &init, double rtol, double atol);
template <typename T>
mm_status dev_step(Plan *p, const double hext[3], unsigned terms, double rtol, double atol,
                   bool relax, bool renorm);
template <typename T>
T *dev_state(Plan *p);
// Copy the device-controlled run's state (rounded to the plan's precision)
// into out on the plan's stream.
hipError_t dev_result(Plan *p, void *out);
// Extra device bytes of the double state of an FP32 plan of this grid.
size_t state64_bytes(const int grid[3]);

hipError_t debug_kernel(Plan &p, int s, double *out);
template <typename T>
hipError_t debug_spectrum(Plan &p, int s, double *out);

}  // namespace mmx
