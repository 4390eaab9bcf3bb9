// kernels.hip -- device pipeline of the micromagnetic hot path on gfx950.
//
// Effective field (Sec. 4) at a state m, one pass per arrow:
//
//   m --F1--> S1 --F2--> S2 --F3--> S2 --I2--> S1 --I1--> h (+ dm/dt)
//
//   F1  x real-to-complex FFT of M = Ms m with the zero padding implied
//       (only nx of Px inputs are loaded), per x-row.
//   F2  y forward FFT (ny of Py inputs nonzero), batched over adjacent kx
//       columns so every global access is a contiguous run of columns.
//   F3  z forward FFT, product with the real symmetric 3x3 spectral kernel
//       (Sec. 4.4: h = N * M becomes a pointwise product after the
//       transform), z inverse FFT, keep k < nz -- one kernel, in registers.
//   I2  y inverse FFT, keep j < ny.
//   I1  x complex-to-real FFT, keep i < nx, then in the same kernel the local
//       terms: exchange stencil with dm/dn = 0 (Sec. 4.2), uniaxial
//       anisotropy (Sec. 4.1), Zeeman, and optionally the LLG right-hand side
//       (Sec. 3, Eq. llg) and the torque maximum used by relaxation.
//
// With a single layer (Pz = 1) F2/F3/I2 collapse into one kernel (y forward,
// product, y inverse).  The 1/(Px Py Pz) of the inverse transform is folded
// into the resident spectral kernel.  No MFMA: FFTs and stencils are not dense
// contractions; everything here is VALU + LDS, bounded by HBM traffic.
#include <cstring>

#include "passes.h"

namespace mmx {

MMX_PASS_INST(extern, float)
MMX_PASS_INST(extern, double)
MMX_MID_INST(extern, float)
MMX_MID_INST(extern, double)

extern template hipError_t launch_local_ext<float>(const Plan&, int, const float*, float*, float*,
                                                  const LocalParams&, double*, bool, int);
extern template hipError_t launch_local_ext<double>(const Plan&, int, const double*, double*,
                                                   double*, const LocalParams&, double*, bool, int);

// ---------------------------------------------------------------------------
// Small vector kernels and deterministic reductions.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 512;
constexpr int kErrBlocks = 2048;  // error norm: 2 kErrBlocks partials <= kRedSlots
static_assert(2 * kErrBlocks <= kRedSlots, "error-norm partials exceed the reduction buffer");

__device__ inline double block_sum(double v)
{
    __shared__ double wsum[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x / 64, l = threadIdx.x & 63;
    if (l == 0) wsum[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) s += wsum[i];
    }
    __syncthreads();
    return s;  // valid in thread 0
}

// out[slot] = sum over partials[0..n) in a fixed order (one block).
__global__ void k_final_sum(const double* __restrict__ partials, int n, double* out, int slot,
                            double scale, int do_sqrt)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += partials[i];
    v = block_sum(v);
    if (threadIdx.x == 0) {
        v *= scale;
        out[slot] = do_sqrt ? sqrt(v) : v;
    }
}

__device__ void dp_control_one(DevCtl* c, const double* red);

// The error norm's two final sums in one launch: block b (a request of a
// batch) sums partials[b pstride .. + n) (squared scaled errors) into
// out[b ostride] as sqrt(scale * sum) and partials[b pstride + n .. + n)
// (non-finite counts) into out[b ostride + 5], each in a fixed order (a
// strided sum per thread, a wavefront tree, the wavefronts in order); with
// ctl, then runs the step controller ctl[b] on them.
constexpr int kSumBlock = 1024;  // threads of k_err_sums (up to 32768 partial pairs)

__global__ __launch_bounds__(kSumBlock) void k_err_sums(const double* __restrict__ partials, int n,
                                                        long pstride, double* out, long ostride,
                                                        double scale, DevCtl* ctl)
{
    __shared__ double ws[2][kSumBlock / 64];
    partials += (long)blockIdx.x * pstride;
    out += (long)blockIdx.x * ostride;
    double v = 0.0, w = 0.0;
    for (int i = threadIdx.x; i < n; i += kSumBlock) {
        v += partials[i];
        w += partials[n + i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_down(v, off, 64);
        w += __shfl_down(w, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        ws[0][threadIdx.x / 64] = v;
        ws[1][threadIdx.x / 64] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v = w = 0.0;
        for (int i = 0; i < kSumBlock / 64; ++i) {
            v += ws[0][i];
            w += ws[1][i];
        }
        out[0] = sqrt(v * scale);
        out[5] = w;
        // the step controller of request b (ctl: device-controlled steps)
        if (ctl) dp_control_one(ctl + blockIdx.x, out);
    }
}

// p[i * stride] = v for i < n.
__global__ void k_fill_strided(double* p, int n, long stride, double v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[(long)i * stride] = v;
}

__global__ void k_fill(double* p, int n, double v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Coefficients of a stage combination.  h: if not null, every coefficient is
// multiplied by *h (the step size held on the device by the device-side
// controller); the host-driven path folds h into c and leaves h null.  In a
// batch (blockIdx.y = request) request b's step size is h[b * hstride].
struct Coef7 {
    double c[7];
    const double* h;
    long hstride;
};
static_assert(sizeof(DevCtl) % sizeof(double) == 0, "controller records are whole doubles");
constexpr long kCtlStride = sizeof(DevCtl) / sizeof(double);

template <typename T>
struct Ptr7 {
    const T* p[7];
};

// 16-byte vectors for the Runge-Kutta vector kernels.
template <typename T>
struct V16;
template <>
struct V16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct V16<double> {
    using type = double2;
    static constexpr int n = 2;
};

template <typename T>
__device__ inline void vload(const T* p, T (&o)[V16<T>::n])
{
    typename V16<T>::type v = *reinterpret_cast<const typename V16<T>::type*>(p);
    if constexpr (V16<T>::n == 4) {
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else {
        o[0] = v.x; o[1] = v.y;
    }
}
template <typename T>
__device__ inline void vstore(T* p, const T (&o)[V16<T>::n])
{
    typename V16<T>::type v;
    if constexpr (V16<T>::n == 4) {
        v.x = o[0]; v.y = o[1]; v.z = o[2]; v.w = o[3];
    } else {
        v.x = o[0]; v.y = o[1];
    }
    *reinterpret_cast<typename V16<T>::type*>(p) = v;
}

// y_out = y + sum_{j < NK} c_j k_j.  VEC: every pointer is 16-byte aligned and
// n3 is a multiple of the vector width.
template <typename T, int NK, bool VEC>
__global__ __launch_bounds__(kBlock) void k_rk_combine(T* __restrict__ y_out,
                                                       const T* __restrict__ y, Coef7 cf,
                                                       Ptr7<T> ks, long n3)
{
    constexpr int W = VEC ? V16<T>::n : 1;
    // request blockIdx.y of a batch: its vectors follow those of the previous one
    const long bo = (long)blockIdx.y * n3;
    y_out += bo;
    y += bo;
#pragma unroll
    for (int j = 0; j < NK; ++j) ks.p[j] += bo;
    const double hs = cf.h ? cf.h[blockIdx.y * cf.hstride] : 1.0;
    T cj[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) cj[j] = (T)(cf.c[j] * hs);
    const long nv = n3 / W;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
         q += (long)gridDim.x * blockDim.x) {
        T acc[W];
        if constexpr (VEC) vload(y + q * W, acc); else acc[0] = y[q];
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            if (cf.c[j] == 0.0) continue;
            T kv[W];
            if constexpr (VEC) vload(ks.p[j] + q * W, kv); else kv[0] = ks.p[j][q];
#pragma unroll
            for (int w = 0; w < W; ++w) acc[w] += cj[j] * kv[w];
        }
        if constexpr (VEC) vstore(y_out + q * W, acc); else y_out[q] = acc[0];
    }
}

// Sum over magnetic components of (e/sc)^2 with e = sum_j c_j k_j (in double)
// and sc = atol + rtol max(|y|, |y1|); also counts non-finite entries of y.
template <typename T, bool VEC, bool PERCELL>
__global__ __launch_bounds__(kBlock) void k_err_norm(const T* __restrict__ y,
                                                     const T* __restrict__ y1, Coef7 cf, Ptr7<T> ks,
                                                     long N, const T* __restrict__ Ms_cell,
                                                     double rtol, double atol, double* partials)
{
    constexpr int W = VEC ? V16<T>::n : 1;
    // request blockIdx.y of a batch (uniform material, no Ms_cell): its
    // vectors and its 2 gridDim.x partials follow those of the previous one
    const long bo = (long)blockIdx.y * 3 * N;
    y += bo;
    y1 += bo;
#pragma unroll
    for (int j = 0; j < 7; ++j) ks.p[j] += bo;
    partials += (long)blockIdx.y * 2 * gridDim.x;
    const double hs = cf.h ? cf.h[blockIdx.y * cf.hstride] : 1.0;
    double cj[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) cj[j] = cf.c[j] * hs;
    double acc = 0.0, bad = 0.0;
    const long nv = 3 * N / W;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
         q += (long)gridDim.x * blockDim.x) {
        T a[W], b[W], ms[W];
        if constexpr (VEC) {
            vload(y + q * W, a);
            vload(y1 + q * W, b);
        } else {
            a[0] = y[q];
            b[0] = y1[q];
        }
        if constexpr (PERCELL) {
            // W divides N, so a vector never straddles two components
            const long cell = (q * W) % N;
            if constexpr (VEC) vload(Ms_cell + cell, ms); else ms[0] = Ms_cell[cell];
        }
        double e[W];
#pragma unroll
        for (int w = 0; w < W; ++w) e[w] = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            if (cf.c[j] == 0.0) continue;
            T kv[W];
            if constexpr (VEC) vload(ks.p[j] + q * W, kv); else kv[0] = ks.p[j][q];
#pragma unroll
            for (int w = 0; w < W; ++w) e[w] += cj[j] * (double)kv[w];
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (!isfinite((double)a[w])) bad += 1.0;
            if (PERCELL && ms[w] == (T)0) continue;
            const double ya = fabs((double)a[w]), yb = fabs((double)b[w]);
            const double sc = atol + rtol * (ya > yb ? ya : yb);
            const double r = e[w] / sc;
            acc += r * r;
        }
    }
    acc = block_sum(acc);
    bad = block_sum(bad);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = acc;
        partials[gridDim.x + blockIdx.x] = bad;
    }
}

template <typename T>
__global__ void k_renorm(T* __restrict__ m, const T* __restrict__ Ms_cell, long N)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        if (Ms_cell && Ms_cell[q] == (T)0) {
            m[q] = m[N + q] = m[2 * N + q] = (T)0;
            continue;
        }
        const T x = m[q], y = m[N + q], z = m[2 * N + q];
        const T inv = (T)1 / sqrt(x * x + y * y + z * z);
        m[q] = x * inv;
        m[N + q] = y * inv;
        m[2 * N + q] = z * inv;
    }
}

// ---------------------------------------------------------------------------
// Device-side Dormand-Prince control (single-thread kernels on DevCtl).  The
// rules are those of the host-driven loop: accept iff err <= 1, factor
// min(10, max(0.2, 0.9 err^-1/5)) (no growth right after a rejection, a step
// clipped to t_end keeps the proposal), a non-finite trial error is a
// rejection with factor 0.2 unless the state itself is non-finite.
// ---------------------------------------------------------------------------
__global__ void k_dp_begin(DevCtl* c, const double* __restrict__ red, int nbatch, int rstride)
{
    // one thread per request of a batch, its reductions rstride doubles apart
    if ((int)threadIdx.x >= nbatch) return;
    c += threadIdx.x;
    if (c->done) return;
    // a relaxation's torque at its current state: the maximum the previous
    // step's closing evaluation (or the start) left in red[1]
    if (c->relax) c->torque = red[(long)threadIdx.x * rstride + 1];
    if (c->relax && c->torque < c->torque_tol) {
        c->done = 1;
        c->result = MM_OK;
    } else if (c->accepted >= c->max_steps) {
        c->done = 1;
        c->result = c->relax ? MM_ENOTCONV : MM_OK;
    } else if (!(c->t < c->t_end)) {
        c->done = 1;
        c->result = MM_OK;
    }
    if (c->done) {
        c->h = 0.0;  // the rest of the step leaves every buffer that matters unchanged
        return;
    }
    double h = c->dt;
    if (c->t + h > c->t_end) h = c->t_end - c->t;
    c->h = h;
}

// Accept or reject one request's step from its error norm red[0] (red[5]:
// non-finite entries of the state) and choose the next step size.
__device__ void dp_control_one(DevCtl* c, const double* red)
{
    c->commit = 0;
    if (c->done) return;
    c->rhs_evals += 6;
    double err = red[0];
    c->err_last = err;
    const double h = c->h;
    if (!isfinite(err)) {
        if (red[5] != 0.0) {
            c->done = 1;
            c->result = MM_ENONFINITE;
            return;
        }
        err = HUGE_VAL;
    }
    if (err <= 1.0) {
        c->t += h;
        c->accepted++;
        c->commit = 1;
        if (c->renorm) c->rhs_evals += 1;
        double fac = err == 0.0 ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * pow(err, -0.2)));
        if (c->last_rejected && fac > 1.0) fac = 1.0;
        if (!(h < c->dt)) c->dt = fac * h;
        c->last_rejected = 0;
    } else {
        c->rejected++;
        c->dt = fmax(0.2, 0.9 * pow(err, -0.2)) * h;
        c->last_rejected = 1;
    }
    if (c->dt < c->dt_min) {
        c->done = 1;
        c->result = MM_EDTMIN;
    }
}

__global__ void k_dp_torque(DevCtl* c, const double* __restrict__ red, int nbatch, int rstride)
{
    if ((int)threadIdx.x >= nbatch) return;
    c += threadIdx.x;
    red += (long)threadIdx.x * rstride;
    if (!c->done) c->torque = red[1];
}

// y = y1 (renormalised on magnetic cells, zero on vacuum cells, when
// c->renorm) and k0 = k6 (without renorm), on acceptance only.
template <typename T>
__global__ void k_dp_commit(const DevCtl* __restrict__ c, T* __restrict__ y,
                            const T* __restrict__ y1, T* __restrict__ k0,
                            const T* __restrict__ k6, const T* __restrict__ Ms_cell, long N)
{
    // request blockIdx.y of a batch: its controller and vectors
    const long bo = (long)blockIdx.y * 3 * N;
    c += blockIdx.y;
    y += bo;
    y1 += bo;
    k0 += bo;
    k6 += bo;
    if (!c->commit) return;
    const bool renorm = c->renorm != 0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        T x = y1[q], yy = y1[N + q], z = y1[2 * N + q];
        if (renorm) {
            if (Ms_cell && Ms_cell[q] == (T)0) {
                x = yy = z = (T)0;
            } else {
                const T inv = (T)1 / sqrt(x * x + yy * yy + z * z);
                x *= inv;
                yy *= inv;
                z *= inv;
            }
        } else {
            k0[q] = k6[q];
            k0[N + q] = k6[N + q];
            k0[2 * N + q] = k6[2 * N + q];
        }
        y[q] = x;
        y[N + q] = yy;
        y[2 * N + q] = z;
    }
}

// Anisotropy energy density summed over magnetic cells (per block, in
// double): -Ku1 (e.m)^2 - Ku2 (e.m)^4 + Kc1 (m1^2 m2^2 + m2^2 m3^2 + m3^2 m1^2)
// + Kc2 m1^2 m2^2 m3^2, m_i along the cubic axes.
struct AnisE {
    double ku1, ku2, kc1, kc2;
    double eu[3];
    double ec[3][3];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_anis_energy(const T* __restrict__ m,
                                                        const T* __restrict__ Ms_cell, double Ms,
                                                        long N, AnisE A, double* partials,
                                                        const double* __restrict__ lw, long nxy,
                                                        const T* __restrict__ Ku_cell)
{
    double acc = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        const double ms = Ms_cell ? (double)Ms_cell[q] : Ms;
        if (ms == 0.0) continue;
        const double mx = m[q], my = m[N + q], mz = m[2 * N + q];
        const double em = A.eu[0] * mx + A.eu[1] * my + A.eu[2] * mz;
        double pr[3];
        for (int a = 0; a < 3; ++a) pr[a] = A.ec[a][0] * mx + A.ec[a][1] * my + A.ec[a][2] * mz;
        const double q0 = pr[0] * pr[0], q1 = pr[1] * pr[1], q2 = pr[2] * pr[2];
        const double ku1 = Ku_cell ? (double)Ku_cell[q] : A.ku1;
        acc += (lw ? lw[q / nxy] : 1.0) *
               (-ku1 * em * em - A.ku2 * em * em * em * em +
                A.kc1 * (q0 * q1 + q1 * q2 + q2 * q0) + A.kc2 * q0 * q1 * q2);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot_ms(const T* __restrict__ a, const T* __restrict__ b,
                                                   const T* __restrict__ Ms_cell, double Ms,
                                                   long N, double* partials,
                                                   const double* __restrict__ lw, long nxy)
{
    double acc = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        const double ms = (Ms_cell ? (double)Ms_cell[q] : Ms) * (lw ? lw[q / nxy] : 1.0);
        acc += ms * ((double)a[q] * b[q] + (double)a[N + q] * b[N + q] +
                     (double)a[2 * N + q] * b[2 * N + q]);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_norms(const T* __restrict__ y,
                                                        const T* __restrict__ f0,
                                                        const T* __restrict__ f1,
                                                        const T* __restrict__ Ms_cell, long N,
                                                        double rtol, double atol,
                                                        double* partials)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < 3 * N;
         q += (long)gridDim.x * blockDim.x) {
        if (Ms_cell && Ms_cell[q % N] == (T)0) continue;
        const double sc = atol + rtol * fabs((double)y[q]);
        const double a = (double)y[q] / sc, b = (double)f0[q] / sc;
        s0 += a * a;
        s1 += b * b;
        if (f1) {
            const double c = ((double)f1[q] - (double)f0[q]) / sc;
            s2 += c * c;
        }
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    s2 = block_sum(s2);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s0;
        partials[kRedBlocks + blockIdx.x] = s1;
        partials[2 * kRedBlocks + blockIdx.x] = s2;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_count_mag(const T* __restrict__ Ms_cell, long N,
                                                      double* partials)
{
    double acc = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x)
        acc += Ms_cell[q] != (T)0 ? 1.0 : 0.0;
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Numbers of negative and of positive entries of v[0..N) into partials
// [0, kRedBlocks) and [kRedBlocks, 2 kRedBlocks).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_count_signs(const T* __restrict__ v, long N,
                                                        double* partials)
{
    double neg = 0.0, pos = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        neg += v[q] < (T)0 ? 1.0 : 0.0;
        pos += v[q] > (T)0 ? 1.0 : 0.0;
    }
    neg = block_sum(neg);
    pos = block_sum(pos);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = neg;
        partials[kRedBlocks + blockIdx.x] = pos;
    }
}

// ---------------------------------------------------------------------------
// Differentiation (inverse design).  The effective field is h = H m + h_zee
// with H the demag (K Ms m), exchange (diag(2/(mu0 Ms)) A~ m) and anisotropy
// parts; K is symmetric and even, A~ symmetric, so
//   H^T z = Ms (K z) + A~ (2 z/(mu0 Ms)) + (2 Ku/(mu0 Ms)) e (e.z)
// and at fixed m, d(z.h)/dMs = m.(K z) - 2/(mu0 Ms^2) z.(A~ m)
//                              - 2 Ku/(mu0 Ms^2) (e.z)(e.m).
// For the LLG right-hand side f = -g' [m x h + alpha m x (m x h)] and a
// cotangent w:  d(w.f)/dm|_h = -g' [h x w + alpha (w (m.h) + h (w.m) - 2 m (w.h))]
//               z = d(w.f)/dh = -g' [w x m + alpha (m (w.m) - w |m|^2)].
// ---------------------------------------------------------------------------
// g (may be null: then z is w masked to magnetic cells) and z per cell.
template <typename T, bool PERCELL>
__global__ void k_vjp_pre(const T* __restrict__ m, const T* __restrict__ h,
                          const T* __restrict__ w, const T* __restrict__ Ms_cell, T Ms, long N,
                          T gp, T alpha, T* __restrict__ g_out, T* __restrict__ z_out)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        const T ms = PERCELL ? Ms_cell[q] : Ms;
        const T wx = w[q], wy = w[N + q], wz = w[2 * N + q];
        if (ms == (T)0) {
            z_out[q] = z_out[N + q] = z_out[2 * N + q] = (T)0;
            if (g_out) g_out[q] = g_out[N + q] = g_out[2 * N + q] = (T)0;
            continue;
        }
        if (!g_out) {
            z_out[q] = wx;
            z_out[N + q] = wy;
            z_out[2 * N + q] = wz;
            continue;
        }
        const T mx = m[q], my = m[N + q], mz = m[2 * N + q];
        const T hx = h[q], hy = h[N + q], hz = h[2 * N + q];
        const T mh = mx * hx + my * hy + mz * hz, wm = wx * mx + wy * my + wz * mz;
        const T wh = wx * hx + wy * hy + wz * hz, mm = mx * mx + my * my + mz * mz;
        g_out[q] = -gp * ((hy * wz - hz * wy) + alpha * (wx * mh + hx * wm - (T)2 * mx * wh));
        g_out[N + q] = -gp * ((hz * wx - hx * wz) + alpha * (wy * mh + hy * wm - (T)2 * my * wh));
        g_out[2 * N + q] = -gp * ((hx * wy - hy * wx) + alpha * (wz * mh + hz * wm - (T)2 * mz * wh));
        z_out[q] = -gp * ((wy * mz - wz * my) + alpha * (mx * wm - wx * mm));
        z_out[N + q] = -gp * ((wz * mx - wx * mz) + alpha * (my * wm - wy * mm));
        z_out[2 * N + q] = -gp * ((wx * my - wy * mx) + alpha * (mz * wm - wz * mm));
    }
}

struct AdjParams {
    int nx, ny, nz;
    long N;
    long s1_comp;
    int Hxp;
    int with_demag, with_exch, with_anis;
    double Ms;
    double exch;  // 2 A / mu0
    double idx2, idy2, idz2;
    double anis;  // 2 Ku / mu0
    double eu[3];
};

// nu = g + H^T z (x inverse transform of the spectrum of K z in S1, then the
// transposed local terms); gms += d(z.h)/dMs (double, may be null).
template <typename T, int M, bool PERCELL>
__global__ __launch_bounds__((XC2R<T, M>::kRows * 3 * XC2R<T, M>::kT)) void k_adj_local(
    const cx<T>* __restrict__ S1, const T* __restrict__ m, const T* __restrict__ z,
    const T* __restrict__ g, const T* __restrict__ Ms_cell, AdjParams P, T* __restrict__ nu,
    double* __restrict__ gms, int njt, long nblocks, const cx<T>* __restrict__ tw, int Lmax)
{
    using G = XC2R<T, M>;
    constexpr int kRows = G::kRows, kL = G::kL;
    __shared__ cx<T> lds[kRows * 3 * kL];
    const long lb = xcd_logical();
    if (lb >= nblocks) return;
    const int k = MMX_X1_KFAST ? (int)(lb % P.nz) : (int)(lb / njt);
    const int j0 = (MMX_X1_KFAST ? (int)(lb / P.nz) : (int)(lb % njt)) * kRows;
    const int nx = P.nx, ny = P.ny;
    if (P.with_demag) x_c2r_rows<T, M>(S1, lds, k, j0, ny, P.s1_comp, P.Hxp, tw, Lmax);
    const long N = P.N;
    const T exch = (T)P.exch, anis = (T)P.anis;
    const T ix2 = (T)P.idx2, iy2 = (T)P.idy2, iz2 = (T)P.idz2;
    const T eux = (T)P.eu[0], euy = (T)P.eu[1], euz = (T)P.eu[2];
    for (int idx = threadIdx.x; idx < kRows * nx; idx += blockDim.x) {
        const int rl = idx / nx, i = idx - rl * nx;
        const int j = j0 + rl;
        if (j >= ny) continue;
        const long cell = i + (long)nx * (j + (long)ny * k);
        const T ms = PERCELL ? Ms_cell[cell] : (T)P.Ms;
        const T mx = m[cell], my = m[N + cell], mz = m[2 * N + cell];
        T nx_ = g ? g[cell] : (T)0, ny_ = g ? g[N + cell] : (T)0, nz_ = g ? g[2 * N + cell] : (T)0;
        double dms = 0.0;
        if (P.with_demag) {
            const T kx = x_c2r_value<T, M>(S1, lds, rl, 0, i, k, j, ny, P.s1_comp, P.Hxp);
            const T ky = x_c2r_value<T, M>(S1, lds, rl, 1, i, k, j, ny, P.s1_comp, P.Hxp);
            const T kz = x_c2r_value<T, M>(S1, lds, rl, 2, i, k, j, ny, P.s1_comp, P.Hxp);
            nx_ += ms * kx;
            ny_ += ms * ky;
            nz_ += ms * kz;
            dms += (double)mx * kx + (double)my * ky + (double)mz * kz;
        }
        if (ms != (T)0) {
            const T inv_ms = (T)1 / ms;
            const T zx = z[cell], zy = z[N + cell], zz = z[2 * N + cell];
            if (P.with_exch) {
                // A~ (z / Ms) and A~ m over magnetic neighbours
                T ax = 0, ay = 0, az = 0, lx = 0, ly = 0, lz = 0;
                const T szx = zx * inv_ms, szy = zy * inv_ms, szz = zz * inv_ms;
                auto nb = [&](long q, T w) {
                    const T mq = PERCELL ? Ms_cell[q] : (T)P.Ms;
                    if (mq == (T)0) return;
                    const T iq = (T)1 / mq;
                    ax += w * (z[q] * iq - szx);
                    ay += w * (z[N + q] * iq - szy);
                    az += w * (z[2 * N + q] * iq - szz);
                    lx += w * (m[q] - mx);
                    ly += w * (m[N + q] - my);
                    lz += w * (m[2 * N + q] - mz);
                };
                if (i > 0) nb(cell - 1, ix2);
                if (i + 1 < nx) nb(cell + 1, ix2);
                if (j > 0) nb(cell - nx, iy2);
                if (j + 1 < ny) nb(cell + nx, iy2);
                if (k > 0) nb(cell - (long)nx * ny, iz2);
                if (k + 1 < P.nz) nb(cell + (long)nx * ny, iz2);
                nx_ += exch * ax;
                ny_ += exch * ay;
                nz_ += exch * az;
                dms -= (double)(exch * inv_ms * inv_ms) * ((double)zx * lx + (double)zy * ly + (double)zz * lz);
            }
            if (P.with_anis) {
                const T ez = eux * zx + euy * zy + euz * zz;
                const T em = eux * mx + euy * my + euz * mz;
                const T ca = anis * inv_ms * ez;
                nx_ += ca * eux;
                ny_ += ca * euy;
                nz_ += ca * euz;
                dms -= (double)(anis * inv_ms * inv_ms) * (double)ez * (double)em;
            }
        }
        nu[cell] = nx_;
        nu[N + cell] = ny_;
        nu[2 * N + cell] = nz_;
        if (gms) gms[cell] += dms;
    }
}

// out = sum_{j < NK} c_j v_j
template <typename T, int NK>
__global__ void k_lincomb(T* __restrict__ out, Coef7 cf, Ptr7<T> v, long n3)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n3;
         q += (long)gridDim.x * blockDim.x) {
        T acc = (T)0;
#pragma unroll
        for (int j = 0; j < NK; ++j) acc += (T)cf.c[j] * v.p[j][q];
        out[q] = acc;
    }
}

// partial sums of m_z over a region mask
template <typename T>
__global__ __launch_bounds__(kBlock) void k_region_mz(const T* __restrict__ m,
                                                      const unsigned char* __restrict__ region,
                                                      long N, double* partials)
{
    double acc = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x)
        if (region[q]) acc += (double)m[2 * N + q];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// *out += scale * sum(partials[0..n))
__global__ void k_final_accum(const double* __restrict__ partials, int n, double* out, double scale)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += partials[i];
    v = block_sum(v);
    if (threadIdx.x == 0) *out += scale * v;
}

// lam_z += val on the region
template <typename T>
__global__ void k_add_region(T* __restrict__ lam, const unsigned char* __restrict__ region, long N,
                             T val)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x)
        if (region[q]) lam[2 * N + q] += val;
}

template <typename T>
__global__ void k_from_double(const double* __restrict__ in, T* __restrict__ out, long n)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        out[q] = (T)in[q];
}

__global__ void k_zero_d(double* __restrict__ p, long n)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

template <typename T, int M, bool PC>
static hipError_t launch_adj_M(const Plan& p, const T* m, const T* z, const T* g, T* nu,
                               double* gms, const AdjParams& P)
{
    using G = XC2R<T, M>;
    const int njt = (p.n[1] + G::kRows - 1) / G::kRows;
    const long nblocks = (long)njt * p.n[2];
    k_adj_local<T, M, PC><<<xcd_grid(nblocks), G::kRows * 3 * G::kT, 0, p.stream>>>(
        (const cx<T>*)p.S1, m, z, g, (const T*)p.Ms_cell, P, nu, gms, njt, nblocks,
        (const cx<T>*)p.tw, p.Lmax);
    return hipGetLastError();
}

template <typename T, bool PC>
static hipError_t launch_adj(const Plan& p, int M, const T* m, const T* z, const T* g, T* nu,
                             double* gms, const AdjParams& P)
{
    switch (M) {
#define MMX_A(LL) \
    case LL: return launch_adj_M<T, LL, PC>(p, m, z, g, nu, gms, P);
        MMX_A(0) MMX_CASES(MMX_A)
#undef MMX_A
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Demag kernel set-up (once per plan).
// ---------------------------------------------------------------------------
// Near field: -N_Newell for offsets 0 <= I < nI etc., all six components,
// in double-double (rounded to double at the end).
__global__ void k_near(double* __restrict__ near, int nI, int nJ, int nK, double dx, double dy,
                       double dz)
{
    const long total = 6L * nI * nJ * nK;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int s = (int)(q / ((long)nI * nJ * nK));
    const long o = q % ((long)nI * nJ * nK);
    const int I = (int)(o % nI), J = (int)((o / nI) % nJ), K = (int)(o / ((long)nI * nJ));
    near[q] = kernel_near(s, I, J, K, dx, dy, dz);
}

// Place component s into the zero-padded real grid: entry (pi, pj, pk) holds
// K(I, J, K) with I = pi (pi < nx) or pi - Px (pi > Px - nx), else zero.
__global__ void k_place(double* __restrict__ R, int s, int nx, int ny, int nz, int Px, int Py,
                        int Pz, const double* __restrict__ near, int nI, int nJ, int nK, int p,
                        double dx, double dy, double dz)
{
    const long total = (long)Px * Py * Pz;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int pi = (int)(q % Px), pj = (int)((q / Px) % Py), pk = (int)(q / ((long)Px * Py));
    auto off = [](int pp, int n, int P, int& o) {
        if (pp < n) { o = pp; return true; }
        if (pp > P - n) { o = pp - P; return true; }
        return false;
    };
    int I, J, K;
    double v = 0.0;
    if (off(pi, nx, Px, I) && off(pj, ny, Py, J) && off(pk, nz, Pz, K)) {
        const int aI = I < 0 ? -I : I, aJ = J < 0 ? -J : J, aK = K < 0 ? -K : K;
        int cheb = aI > aJ ? aI : aJ;
        cheb = cheb > aK ? cheb : aK;
        if (p < 0 || cheb <= p) {
            double sg = 1.0;
            if (s == 3) sg = ((I < 0) != (J < 0)) ? -1.0 : 1.0;
            if (s == 4) sg = ((I < 0) != (K < 0)) ? -1.0 : 1.0;
            if (s == 5) sg = ((J < 0) != (K < 0)) ? -1.0 : 1.0;
            v = sg * near[(((long)s * nK + aK) * nJ + aJ) * nI + aI];
        } else {
            v = kernel_dipole(s, I, J, K, dx, dy, dz);
        }
    }
    R[q] = v;
}

// Keep the real part of the transformed component (it is real by parity) for
// 0 <= ky <= Py/2, 0 <= kz <= Pz/2, scaled by 1/(Px Py Pz).
template <typename T>
__global__ void k_fold(T* __restrict__ Khat, const cx<double>* __restrict__ C, int Hx, int Hxp,
                       int Py, int Pz, double scale)
{
    const int hy = Py / 2 + 1, hz = Pz / 2 + 1;
    const long total = (long)hz * hy * Hxp;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int kx = (int)(q % Hxp), ky = (int)((q / Hxp) % hy), kz = (int)(q / ((long)Hxp * hy));
    Khat[q] = kx < Hx ? (T)(C[((long)kz * Py + ky) * Hxp + kx].x * scale) : (T)0;
}

#define MMX_TRY_PROF(x)                   \
    do {                                  \
        hipError_t e__ = (x);             \
        if (e__ != hipSuccess) return e__; \
    } while (0)

#define MMX_TRY(x)                        \
    do {                                  \
        hipError_t e__ = (x);             \
        if (e__ != hipSuccess) return e__; \
    } while (0)

static long blocks_for(long n, int bs) { return (n + bs - 1) / bs; }

// ---------------------------------------------------------------------------
// Per-pass event timing (mm_profile).
// ---------------------------------------------------------------------------
static hipError_t take_event(Plan& p, hipEvent_t* e)
{
    if (!p.prof.pool.empty()) {
        *e = p.prof.pool.back();
        p.prof.pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

hipError_t prof_flush(Plan& p)
{
    if (p.prof.pending.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(p.stream);
    if (e != hipSuccess) return e;
    for (auto& r : p.prof.pending) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return e;
        p.prof.ms[r.pass] += ms;
        p.prof.cnt[r.pass] += 1;
        p.prof.pool.push_back(r.a);
        p.prof.pool.push_back(r.b);
    }
    p.prof.pending.clear();
    return hipSuccess;
}

hipError_t prof_begin(Plan& p, int pass, hipEvent_t* a)
{
    (void)pass;
    if (!p.prof.on) return hipSuccess;
    hipError_t e = take_event(p, a);
    if (e != hipSuccess) return e;
    return hipEventRecord(*a, p.stream);
}

hipError_t prof_end(Plan& p, int pass, hipEvent_t a)
{
    if (!p.prof.on) return hipSuccess;
    hipEvent_t b;
    hipError_t e = take_event(p, &b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, p.stream);
    if (e != hipSuccess) return e;
    p.prof.pending.push_back({pass, a, b});
    if (p.prof.pending.size() >= 4096) return prof_flush(p);
    return hipSuccess;
}

// Launch `body` between a pair of profiling events for `pass`.
template <typename F>
static hipError_t timed(Plan& p, int pass, F&& body)
{
    hipEvent_t a = nullptr;
    MMX_TRY_PROF(prof_begin(p, pass, &a));
    MMX_TRY_PROF(body());
    return prof_end(p, pass, a);
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch()
    {
        for (void* q : ptrs) (void)hipFree(q);
    }
    template <typename U>
    hipError_t get(U** out, size_t bytes)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
        if (e != hipSuccess) return e;
        ptrs.push_back(q);
        *out = static_cast<U*>(q);
        return hipSuccess;
    }
};

template <typename T>
hipError_t init_twiddles(Plan& p)
{
    k_twiddles<T><<<blocks_for(p.Lmax, 256), 256, 0, p.stream>>>((cx<T>*)p.tw, p.Lmax);
    return hipGetLastError();
}

static hipError_t near_table(Plan& p, Scratch& sc, double** near, int& nI, int& nJ, int& nK)
{
    const int lim = p.demag_p < 0 ? (1 << 30) : p.demag_p;
    nI = std::min(p.n[0] - 1, lim) + 1;
    nJ = std::min(p.n[1] - 1, lim) + 1;
    nK = std::min(p.n[2] - 1, lim) + 1;
    const long total = 6L * nI * nJ * nK;
    MMX_TRY(sc.get(near, sizeof(double) * total));
    k_near<<<blocks_for(total, 64), 64, 0, p.stream>>>(*near, nI, nJ, nK, p.d[0], p.d[1], p.d[2]);
    return hipGetLastError();
}

hipError_t debug_kernel(Plan& p, int s, double* out)
{
    Scratch sc;
    double* near;
    int nI, nJ, nK;
    MMX_TRY(near_table(p, sc, &near, nI, nJ, nK));
    const long PN = (long)p.P[0] * p.P[1] * p.P[2];
    k_place<<<blocks_for(PN, 256), 256, 0, p.stream>>>(out, s, p.n[0], p.n[1], p.n[2], p.P[0],
                                                      p.P[1], p.P[2], near, nI, nJ, nK,
                                                      p.demag_p, p.d[0], p.d[1], p.d[2]);
    MMX_TRY(hipGetLastError());
    return hipStreamSynchronize(p.stream);
}

// Thin layers: near-field table of K^{ts}(I, J) for 0 <= I < nI, 0 <= J < nJ
// and every layer pair with |t - s| <= p, all six components.
__global__ void k_near_layer(double* __restrict__ near, int nI, int nJ, int nz,
                             const double* __restrict__ zb, double dx, double dy, int p)
{
    const long per = (long)nz * nz * nJ * nI;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 6 * per) return;
    const int comp = (int)(q / per);
    const long o = q % per;
    const int I = (int)(o % nI), J = (int)((o / nI) % nJ);
    const int ts = (int)(o / ((long)nI * nJ));
    const int t = ts / nz, s = ts % nz;
    const int dts = t > s ? t - s : s - t;
    near[q] = (p < 0 || dts <= p) ? kernel_near_layer(comp, I, J, zb, t, s, dx, dy) : 0.0;
}

// Place K^{ts}_comp into the zero-padded lateral grid (Px x Py).
__global__ void k_place_layer(double* __restrict__ R, int comp, int t, int s, int nx, int ny,
                              int nz, int Px, int Py, const double* __restrict__ near, int nI,
                              int nJ, const double* __restrict__ zb, int p, double dx, double dy)
{
    const long total = (long)Px * Py;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int pi = (int)(q % Px), pj = (int)(q / Px);
    auto off = [](int pp, int n, int P, int& o) {
        if (pp < n) { o = pp; return true; }
        if (pp > P - n) { o = pp - P; return true; }
        return false;
    };
    int I, J;
    double v = 0.0;
    if (off(pi, nx, Px, I) && off(pj, ny, Py, J)) {
        const int aI = I < 0 ? -I : I, aJ = J < 0 ? -J : J, dts = t > s ? t - s : s - t;
        int cheb = aI > aJ ? aI : aJ;
        cheb = cheb > dts ? cheb : dts;
        if (p < 0 || cheb <= p) {
            // lateral mirror symmetry: xy odd in x and y, xz odd in x, yz odd in y
            double sg = 1.0;
            if (comp == 3) sg = ((I < 0) != (J < 0)) ? -1.0 : 1.0;
            if (comp == 4) sg = I < 0 ? -1.0 : 1.0;
            if (comp == 5) sg = J < 0 ? -1.0 : 1.0;
            v = sg * near[(((long)comp * nz + t) * nz + s) * nJ * nI + (long)aJ * nI + aI];
        } else {
            v = kernel_dipole_layer(comp, I, J, zb, t, s, dx, dy);
        }
    }
    R[q] = v;
}

// Keep ky <= Py/2 of the lateral transform of one layer pair, scaled by
// 1/(Px Py): the real part for xx, yy, zz, xy, the imaginary part for xz, yz
// (odd in x only, so their transform is imaginary).
template <typename T>
__global__ void k_fold_layer(T* __restrict__ Khat, const cx<double>* __restrict__ C, int Hx,
                             int Hxp, int Py, int imag, double scale)
{
    const int hy = Py / 2 + 1;
    const long total = (long)hy * Hxp;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int kx = (int)(q % Hxp), ky = (int)(q / Hxp);
    const cx<double> c = C[(long)ky * Hxp + kx];
    Khat[q] = kx < Hx ? (T)((imag ? c.y : c.x) * scale) : (T)0;
}

// Thin layers: mean layer height, the unit of the weights w_t = c_t / c_ref
// of the stored layer-pair kernels.
static double layer_ref(const Plan& p) { return (p.zb.back() - p.zb.front()) / p.n[2]; }

// Packed index of the unordered layer pair a <= b (row-major upper triangle).
__host__ __device__ inline long layer_pair(int a, int b, int nz)
{
    return (long)a * nz - (long)a * (a - 1) / 2 + (b - a);
}

// The layer-pair kernels satisfy reciprocity, V_t N^{ts}(r) = V_s N^{st}(-r)
// (the target average of the field of a uniform source cell, N even in r; it
// holds term by term for the near field and for the dipole far field), so in
// the lateral spectrum W^{ts} = w_t K^^{ts} is Hermitian in (t, s): the real
// xx, yy, zz, xy parts are symmetric and the imaginary xz, yz parts
// antisymmetric.  Only W^{ts} with t <= s is built and stored.
template <typename T>
static hipError_t build_tensor_layers(Plan& p)
{
    Scratch sc;
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int lim = p.demag_p < 0 ? (1 << 30) : p.demag_p;
    const int nI = std::min(nx - 1, lim) + 1, nJ = std::min(ny - 1, lim) + 1;
    const int Px = p.P[0], Py = p.P[1];
    const long PN = (long)Px * Py;
    double *zb, *near, *R;
    cx<double>* C;
    cx<double>* tw64;
    MMX_TRY(sc.get(&zb, sizeof(double) * (nz + 1)));
    MMX_TRY(hipMemcpyAsync(zb, p.zb.data(), sizeof(double) * (nz + 1), hipMemcpyHostToDevice,
                           p.stream));
    const long ntab = 6L * nz * nz * nJ * nI;
    MMX_TRY(sc.get(&near, sizeof(double) * ntab));
    k_near_layer<<<blocks_for(ntab, 64), 64, 0, p.stream>>>(near, nI, nJ, nz, zb, p.d[0], p.d[1],
                                                          p.demag_p);
    MMX_TRY(hipGetLastError());
    MMX_TRY(sc.get(&R, sizeof(double) * PN));
    MMX_TRY(sc.get(&C, sizeof(cx<double>) * (long)Py * p.Hxp));
    MMX_TRY(sc.get(&tw64, sizeof(cx<double>) * p.Lmax));
    k_twiddles<double><<<blocks_for(p.Lmax, 256), 256, 0, p.stream>>>(tw64, p.Lmax);
    MMX_TRY(hipGetLastError());
    Plan q = p;
    q.batch = 1;  // set-up and single-request helpers never run batched
    q.Ms_b = q.Pb = nullptr;
    q.tw = tw64;
    const long hyx = (long)(Py / 2 + 1) * p.Hxp;
    const double cref = layer_ref(p);
    for (int comp = 0; comp < 6; ++comp)
        for (int t = 0; t < nz; ++t)
            for (int s = t; s < nz; ++s) {
                const double wt = (p.zb[t + 1] - p.zb[t]) / cref;
                k_place_layer<<<blocks_for(PN, 256), 256, 0, p.stream>>>(
                    R, comp, t, s, nx, ny, nz, Px, Py, near, nI, nJ, zb, p.demag_p, p.d[0], p.d[1]);
                MMX_TRY(hipGetLastError());
                MMX_TRY((launch_x_r2c<double, false>(q, Px / 2, R, Px, 0, Px, nullptr, 1.0, C,
                                                     p.Hxp, 0, Py, 1)));
                if (Py > 1)
                    MMX_TRY((launch_strided<double, -1>(q, Py, C, C, Py, Py, p.Hxp, p.Hxp, p.Hx, 1,
                                                        0, 0, 1, 0, 0)));
                k_fold_layer<T><<<blocks_for(hyx, 256), 256, 0, p.stream>>>(
                    (T*)p.Khat + comp * p.Kn + layer_pair(t, s, nz) * hyx, C, p.Hx, p.Hxp, Py,
                    comp >= 4 ? 1 : 0, wt / (double)PN);
                MMX_TRY(hipGetLastError());
            }
    return hipStreamSynchronize(p.stream);
}

template <typename T>
hipError_t build_tensor(Plan& p)
{
    if (p.layered) return build_tensor_layers<T>(p);
    Scratch sc;
    double* near;
    int nI, nJ, nK;
    MMX_TRY(near_table(p, sc, &near, nI, nJ, nK));
    const int Px = p.P[0], Py = p.P[1], Pz = p.P[2];
    const long PN = (long)Px * Py * Pz;
    double* R;
    cx<double>* C;
    cx<double>* tw64;
    MMX_TRY(sc.get(&R, sizeof(double) * PN));
    MMX_TRY(sc.get(&C, sizeof(cx<double>) * (long)Pz * Py * p.Hxp));
    MMX_TRY(sc.get(&tw64, sizeof(cx<double>) * p.Lmax));
    k_twiddles<double><<<blocks_for(p.Lmax, 256), 256, 0, p.stream>>>(tw64, p.Lmax);
    MMX_TRY(hipGetLastError());
    // the FFT launchers read the twiddles from the plan: point them at the
    // double table while the kernel is transformed
    Plan q = p;
    q.batch = 1;  // set-up and single-request helpers never run batched
    q.Ms_b = q.Pb = nullptr;
    q.tw = tw64;
    for (int s = 0; s < 6; ++s) {
        k_place<<<blocks_for(PN, 256), 256, 0, p.stream>>>(R, s, p.n[0], p.n[1], p.n[2], Px, Py, Pz,
                                                          near, nI, nJ, nK, p.demag_p, p.d[0],
                                                          p.d[1], p.d[2]);
        MMX_TRY(hipGetLastError());
        // x: real rows of length Px -> Hx bins
        MMX_TRY((launch_x_r2c<double, false>(q, Px / 2, R, Px, 0, Px, nullptr, 1.0, C, p.Hxp, 0,
                                             Py * Pz, 1)));
        // y: in place, pencils along ky (stride Hxp), groups kz
        if (Py > 1)
            MMX_TRY((launch_strided<double, -1>(q, Py, C, C, Py, Py, p.Hxp, p.Hxp, p.Hx, 1, 0, 0,
                                                Pz, (long)Py * p.Hxp, (long)Py * p.Hxp)));
        // z: in place, pencils along kz (stride Py Hxp), groups ky
        if (Pz > 1)
            MMX_TRY((launch_strided<double, -1>(q, Pz, C, C, Pz, Pz, (long)Py * p.Hxp,
                                                (long)Py * p.Hxp, p.Hx, 1, 0, 0, Py, p.Hxp,
                                                p.Hxp)));
        k_fold<T><<<blocks_for(p.Kn, 256), 256, 0, p.stream>>>(
            (T*)p.Khat + s * p.Kn, C, p.Hx, p.Hxp, Py, Pz, 1.0 / (double)PN);
        MMX_TRY(hipGetLastError());
    }
    return hipStreamSynchronize(p.stream);
}

template <typename T>
__global__ void k_to_double(const T* in, double* out, long n, int Hx, int Hxp)
{
    // drop the row padding: (rows x Hxp) -> (rows x Hx)
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const long row = q / Hx, kx = q % Hx;
    out[q] = (double)in[row * Hxp + kx];
}

template <typename T>
hipError_t debug_spectrum(Plan& p, int s, double* out)
{
    const long rows = p.Kn / p.Hxp;
    const long n = rows * p.Hx;
    k_to_double<T><<<blocks_for(n, 256), 256, 0, p.stream>>>((const T*)p.Khat + s * p.Kn, out, n,
                                                            p.Hx, p.Hxp);
    MMX_TRY(hipGetLastError());
    return hipStreamSynchronize(p.stream);
}

// ---------------------------------------------------------------------------
// Thin layers: dense coupling of the layers per lateral frequency,
//   h^_t(kx, ky) = sum_s K^^{ts}(kx, ky) M^_s(kx, ky)
//               = (1 / w_t) sum_s W^{ts}(kx, ky) M^_s(kx, ky),
// in place on the y-transformed spectrum S ([3][nz][Py][Hxp]).  W is stored
// for the layer pairs t <= s only, [6][nz (nz + 1) / 2][Py/2+1][Hxp]: xx, yy,
// zz, xy real, xz, yz imaginary (stored as their imaginary part); a pair
// t > s reads (s, t) with xz, yz negated.  Row Py - ky uses row ky with the
// y-odd components (xy, yz) negated.  A block holds TW consecutive kx of the
// row pair (ky, Py - ky), so every kernel row is read once for both: the
// spectra of all layers of both rows are staged in LDS, then thread (kx, g)
// accumulates targets t = g, g + G, ...; the two targets of a pair run in
// one block, so the second read of a kernel row is a cache hit.
// ---------------------------------------------------------------------------
constexpr int kZdMaxLayers = 16;

template <typename T>
struct ZdTile {
    static constexpr int kTW = sizeof(T) == 4 ? 64 : 32;  // kx per block
};

template <typename T>
__global__ __launch_bounds__(ZdTile<T>::kTW * kZdMaxLayers) void k_zdense(
    cx<T>* __restrict__ S, const T* __restrict__ K, int nz, int Py, int Hx, int Hxp, long s_comp,
    long k_comp, const double* __restrict__ lw, double cref)
{
    constexpr int TW = ZdTile<T>::kTW;
    extern __shared__ unsigned char zd_smem[];
    cx<T>* st = reinterpret_cast<cx<T>*>(zd_smem);  // [row][3][nz][TW]
    const int lane = threadIdx.x % TW, g = threadIdx.x / TW, G = blockDim.x / TW;
    const int kx = blockIdx.x * TW + lane, ky = blockIdx.y, ky2 = Py - ky;
    const bool pair = ky > 0 && 2 * ky < Py;
    const bool valid = kx < Hx;
    const int per_row = 3 * nz;
    for (int r = g; r < (pair ? 2 : 1) * per_row; r += G) {
        const int row = r / per_row, rem = r - row * per_row;
        const int c = rem / nz, k = rem - c * nz;
        const int y = row ? ky2 : ky;
        st[r * TW + lane] = valid ? S[c * s_comp + ((long)k * Py + y) * Hxp + kx] : cx<T>{0, 0};
    }
    __syncthreads();
    if (!valid) return;
    const long hy = Py / 2 + 1;
    for (int t = g; t < nz; t += G) {
        T a[6] = {0, 0, 0, 0, 0, 0}, b[6] = {0, 0, 0, 0, 0, 0};
        for (int sidx = 0; sidx < nz; ++sidx) {
            const bool lower = t > sidx;
            const long kb =
                (layer_pair(lower ? sidx : t, lower ? t : sidx, nz) * hy + ky) * Hxp + kx;
            const T kxx = K[kb], kyy = K[k_comp + kb], kzz = K[2 * k_comp + kb];
            const T kxy = K[3 * k_comp + kb];
            const T vxz = lower ? -K[4 * k_comp + kb] : K[4 * k_comp + kb];
            const T vyz = lower ? -K[5 * k_comp + kb] : K[5 * k_comp + kb];
            // K^ M with the real xx, yy, zz, xy and i v for xz, yz:
            // (i v) M = (-v M.im, v M.re); row Py - ky negates xy and yz
            auto acc = [&](T* h, const cx<T>* Mrow, T sy) {
                const cx<T> Mx = Mrow[sidx * TW], My = Mrow[(nz + sidx) * TW],
                            Mz = Mrow[(2 * nz + sidx) * TW];
                const T cxy = sy * kxy, cyz = sy * vyz;
                h[0] += kxx * Mx.x + cxy * My.x - vxz * Mz.y;
                h[1] += kxx * Mx.y + cxy * My.y + vxz * Mz.x;
                h[2] += cxy * Mx.x + kyy * My.x - cyz * Mz.y;
                h[3] += cxy * Mx.y + kyy * My.y + cyz * Mz.x;
                h[4] += kzz * Mz.x - vxz * Mx.y - cyz * My.y;
                h[5] += kzz * Mz.y + vxz * Mx.x + cyz * My.x;
            };
            acc(a, st + lane, (T)1);
            if (pair) acc(b, st + per_row * TW + lane, (T)-1);
        }
        const T iw = (T)(cref / lw[t]);
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            a[e] *= iw;
            b[e] *= iw;
        }
        const long o = ((long)t * Py + ky) * Hxp + kx;
        S[o] = {a[0], a[1]};
        S[s_comp + o] = {a[2], a[3]};
        S[2 * s_comp + o] = {a[4], a[5]};
        if (pair) {
            const long o2 = ((long)t * Py + ky2) * Hxp + kx;
            S[o2] = {b[0], b[1]};
            S[s_comp + o2] = {b[2], b[3]};
            S[2 * s_comp + o2] = {b[4], b[5]};
        }
    }
}

template <typename T>
static hipError_t launch_zdense(Plan& p, cx<T>* S)
{
    constexpr int TW = ZdTile<T>::kTW;
    const int nz = p.n[2], Py = p.P[1];
    const int G = nz < kZdMaxLayers ? nz : kZdMaxLayers;
    dim3 grid((unsigned)((p.Hx + TW - 1) / TW), (unsigned)(Py / 2 + 1));
    const size_t lds = sizeof(cx<T>) * 2 * 3 * nz * TW;
    k_zdense<T><<<grid, TW * G, lds, p.stream>>>(S, (const T*)p.Khat, nz, Py, p.Hx, p.Hxp,
                                                 (long)nz * Py * p.Hxp, p.Kn, p.lw,
                                                 layer_ref(p));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Field evaluation.
// ---------------------------------------------------------------------------
// Demag convolution up to the x spectrum: S1 <- spectrum of K (Ms src) (or of
// K src with use_ms = false), i.e. every pass but the last inverse x
// transform, which the caller fuses with its local terms.
template <typename T>
static hipError_t demag_to_S1(Plan& p, const T* m, bool use_ms, const StageIn<T>* sc = nullptr)
{
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int Py = p.P[1], Pz = p.P[2];
    const int M = p.P[0] / 2;
    const long s1c = (long)nz * ny * p.Hxp;
    cx<T>* S1 = (cx<T>*)p.S1;
    cx<T>* S2 = (cx<T>*)p.S2;
    const bool pc = p.percell && use_ms;
    const T ms = use_ms ? (T)p.Ms : (T)1;
    // a batch of requests: 3 components each, one after the other; the
    // x forward pass scales by each request's Ms (p.Ms_b)
    const int nc = 3 * p.batch;
    if (p.Pb && (pc || !use_ms || sc || !p.Ms_b || M < 2)) return hipErrorInvalidValue;
    MMX_TRY(timed(p, MM_PASS_X_FWD, [&] {
        return pc ? launch_x_r2c<T, true>(p, M, m, nx, p.N, nx, (const T*)p.Ms_cell, ms, S1, p.Hxp,
                                          s1c, ny * nz, 3, sc)
                  : launch_x_r2c<T, false>(p, M, m, nx, p.N, nx, nullptr, ms, S1, p.Hxp, s1c,
                                           ny * nz, nc, sc);
    }));
    if (p.layered) {
        if (p.Pb) return hipErrorInvalidValue;
        const long s2c = (long)nz * Py * p.Hxp;
        if (Py > 1)
            MMX_TRY(timed(p, MM_PASS_Y_FWD, [&] {
                return launch_strided<T, -1>(p, Py, S1, S2, ny, Py, p.Hxp, p.Hxp, p.Hx, 3, s1c, s2c,
                                             nz, (long)ny * p.Hxp, (long)Py * p.Hxp);
            }));
        MMX_TRY(timed(p, MM_PASS_MID, [&] { return launch_zdense<T>(p, Py > 1 ? S2 : S1); }));
        if (Py > 1)
            MMX_TRY(timed(p, MM_PASS_Y_INV, [&] {
                return launch_strided<T, 1>(p, Py, S2, S1, Py, ny, p.Hxp, p.Hxp, p.Hx, 3, s2c, s1c,
                                            nz, (long)Py * p.Hxp, (long)ny * p.Hxp);
            }));
    } else if (Pz > 1) {
        const long s2c = (long)nz * Py * p.Hxp;
        if (Py > 1)
            MMX_TRY(timed(p, MM_PASS_Y_FWD, [&] {
                return launch_strided<T, -1>(p, Py, S1, S2, ny, Py, p.Hxp, p.Hxp, p.Hx, nc, s1c, s2c,
                                             nz, (long)ny * p.Hxp, (long)Py * p.Hxp);
            }));
        MMX_TRY(timed(p, MM_PASS_MID, [&] {
            return launch_mid<T, 2>(p, Pz, S2, nz, (long)Py * p.Hxp, s2c, p.Hxp, Py);
        }));
        if (Py > 1)
            MMX_TRY(timed(p, MM_PASS_Y_INV, [&] {
                return launch_strided<T, 1>(p, Py, S2, S1, Py, ny, p.Hxp, p.Hxp, p.Hx, nc, s2c, s1c,
                                            nz, (long)Py * p.Hxp, (long)ny * p.Hxp);
            }));
    } else {
        MMX_TRY(timed(p, MM_PASS_MID, [&] { return launch_mid<T, 1>(p, Py, S1, ny, p.Hxp, s1c, 0, 1); }));
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Oersted field (Sec. 4.5): h = sum_s j_s x G(X_t - X_s) as an FFT
// convolution.  G_l is odd along l and even along the other axes, so its
// spectrum is i g with g real, even in ky and kz except for the sign flip of
// g_y for ky > Py/2 and of g_z for kz > Pz/2; the folded octant of g is kept.
// ---------------------------------------------------------------------------
__global__ void k_oe_near(double* __restrict__ near, int nI, int nJ, int nK, double dx, double dy,
                          double dz)
{
    const long per = (long)nI * nJ * nK;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 3 * per) return;
    const int comp = (int)(q / per);
    const long o = q % per;
    const int I = (int)(o % nI), J = (int)((o / nI) % nJ), K = (int)(o / ((long)nI * nJ));
    near[q] = oersted_near(comp, I, J, K, dx, dy, dz);
}

__global__ void k_oe_place(double* __restrict__ R, int comp, int nx, int ny, int nz, int Px, int Py,
                           int Pz, const double* __restrict__ near, int nI, int nJ, int nK, int p,
                           double dx, double dy, double dz)
{
    const long total = (long)Px * Py * Pz;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int pi = (int)(q % Px), pj = (int)((q / Px) % Py), pk = (int)(q / ((long)Px * Py));
    auto off = [](int pp, int n, int P, int& o) {
        if (pp < n) { o = pp; return true; }
        if (pp > P - n) { o = pp - P; return true; }
        return false;
    };
    int I, J, K;
    double v = 0.0;
    if (off(pi, nx, Px, I) && off(pj, ny, Py, J) && off(pk, nz, Pz, K)) {
        const int aI = I < 0 ? -I : I, aJ = J < 0 ? -J : J, aK = K < 0 ? -K : K;
        int cheb = aI > aJ ? aI : aJ;
        cheb = cheb > aK ? cheb : aK;
        if (p < 0 || cheb <= p) {
            const int own = comp == 0 ? I : comp == 1 ? J : K;  // odd along its own axis
            v = (own < 0 ? -1.0 : 1.0) * near[(((long)comp * nK + aK) * nJ + aJ) * nI + aI];
        } else {
            v = oersted_point(comp, I, J, K, dx, dy, dz);
        }
    }
    R[q] = v;
}

template <typename T>
__global__ void k_oe_fold(T* __restrict__ G, const cx<double>* __restrict__ C, int Hx, int Hxp,
                          int Py, int Pz, double scale)
{
    const int hy = Py / 2 + 1, hz = Pz / 2 + 1;
    const long total = (long)hz * hy * Hxp;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int kx = (int)(q % Hxp), ky = (int)((q / Hxp) % hy), kz = (int)(q / ((long)Hxp * hy));
    G[q] = kx < Hx ? (T)(C[((long)kz * Py + ky) * Hxp + kx].y * scale) : (T)0;
}

template <typename T>
static hipError_t oersted_setup(Plan& p)
{
    const int Px = p.P[0], Py = p.P[1], Pz = p.P[2];
    const size_t es = sizeof(T);
    const long gn = (long)(Pz / 2 + 1) * (Py / 2 + 1) * p.Hxp;
    if (p.oe_G) return hipSuccess;
    MMX_TRY(hipMalloc(&p.oe_G, 3 * (size_t)gn * es));
    p.bytes += 3 * (size_t)gn * es;
    Scratch sc;
    const int lim = p.demag_p < 0 ? (1 << 30) : p.demag_p;
    const int nI = std::min(p.n[0] - 1, lim) + 1, nJ = std::min(p.n[1] - 1, lim) + 1,
              nK = std::min(p.n[2] - 1, lim) + 1;
    const long ntab = 3L * nI * nJ * nK;
    double *near, *R;
    cx<double>* C;
    cx<double>* tw64;
    MMX_TRY(sc.get(&near, sizeof(double) * ntab));
    k_oe_near<<<blocks_for(ntab, 64), 64, 0, p.stream>>>(near, nI, nJ, nK, p.d[0], p.d[1], p.d[2]);
    MMX_TRY(hipGetLastError());
    const long PN = (long)Px * Py * Pz;
    MMX_TRY(sc.get(&R, sizeof(double) * PN));
    MMX_TRY(sc.get(&C, sizeof(cx<double>) * (long)Pz * Py * p.Hxp));
    MMX_TRY(sc.get(&tw64, sizeof(cx<double>) * p.Lmax));
    k_twiddles<double><<<blocks_for(p.Lmax, 256), 256, 0, p.stream>>>(tw64, p.Lmax);
    MMX_TRY(hipGetLastError());
    Plan q = p;
    q.batch = 1;  // set-up and single-request helpers never run batched
    q.Ms_b = q.Pb = nullptr;
    q.tw = tw64;
    for (int comp = 0; comp < 3; ++comp) {
        k_oe_place<<<blocks_for(PN, 256), 256, 0, p.stream>>>(R, comp, p.n[0], p.n[1], p.n[2], Px,
                                                             Py, Pz, near, nI, nJ, nK, p.demag_p,
                                                             p.d[0], p.d[1], p.d[2]);
        MMX_TRY(hipGetLastError());
        MMX_TRY((launch_x_r2c<double, false>(q, Px / 2, R, Px, 0, Px, nullptr, 1.0, C, p.Hxp, 0,
                                             Py * Pz, 1)));
        if (Py > 1)
            MMX_TRY((launch_strided<double, -1>(q, Py, C, C, Py, Py, p.Hxp, p.Hxp, p.Hx, 1, 0, 0,
                                                Pz, (long)Py * p.Hxp, (long)Py * p.Hxp)));
        if (Pz > 1)
            MMX_TRY((launch_strided<double, -1>(q, Pz, C, C, Pz, Pz, (long)Py * p.Hxp,
                                                (long)Py * p.Hxp, p.Hx, 1, 0, 0, Py, p.Hxp,
                                                p.Hxp)));
        k_oe_fold<T><<<blocks_for(gn, 256), 256, 0, p.stream>>>((T*)p.oe_G + comp * gn, C, p.Hx,
                                                                p.Hxp, Py, Pz, 1.0 / (double)PN);
        MMX_TRY(hipGetLastError());
    }
    return hipStreamSynchronize(p.stream);
}

template <typename T>
hipError_t oersted_field(Plan& p, const T* j, T* h_out)
{
    MMX_TRY(oersted_setup<T>(p));
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int Py = p.P[1], Pz = p.P[2];
    const long s1c = (long)nz * ny * p.Hxp;
    cx<T>* S1 = (cx<T>*)p.S1;
    cx<T>* S2 = (cx<T>*)p.S2;
    // the demag pass chain with the Oersted product in the last-axis pass
    Plan q = p;
    q.batch = 1;  // set-up and single-request helpers never run batched
    q.Ms_b = q.Pb = nullptr;
    q.Khat = p.oe_G;
    MMX_TRY((launch_x_r2c<T, false>(p, p.P[0] / 2, j, nx, p.N, nx, nullptr, (T)1, S1, p.Hxp, s1c,
                                    ny * nz, 3)));
    if (Pz > 1) {
        const long s2c = (long)nz * Py * p.Hxp;
        if (Py > 1)
            MMX_TRY((launch_strided<T, -1>(p, Py, S1, S2, ny, Py, p.Hxp, p.Hxp, p.Hx, 3, s1c, s2c,
                                           nz, (long)ny * p.Hxp, (long)Py * p.Hxp)));
        MMX_TRY((launch_mid<T, 2, 1>(q, Pz, S2, nz, (long)Py * p.Hxp, s2c, p.Hxp, Py)));
        if (Py > 1)
            MMX_TRY((launch_strided<T, 1>(p, Py, S2, S1, Py, ny, p.Hxp, p.Hxp, p.Hx, 3, s2c, s1c,
                                          nz, (long)Py * p.Hxp, (long)ny * p.Hxp)));
    } else {
        MMX_TRY((launch_mid<T, 1, 1>(q, Py, S1, ny, p.Hxp, s1c, 0, 1)));
    }
    // x inverse: the raw convolution at every cell (uniform Ms 1, no other term)
    LocalParams P{};
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    P.N = p.N;
    P.s1_comp = s1c;
    P.Hxp = p.Hxp;
    P.with_demag = 1;
    P.Ms = 1.0;
    Plan r = p;
    r.percell_A = r.percell_D = r.layered = false;
    return launch_local<T, false, 0>(r, p.P[0] / 2, j, h_out, nullptr, P, nullptr);
}

// The constants of the local pass for plan p at time t (field h_ext, terms,
// alpha_eff and precession of the LLG right-hand side); *ext_out: the
// stencil variant (EXT_* bits) the plan's material needs.
static LocalParams make_local_params(const Plan& p, const double hext[3], unsigned terms, double t,
                                     double alpha_eff, bool precess, int* ext_out)
{
    LocalParams P{};
    P.nx = p.n[0];
    P.ny = p.n[1];
    P.nz = p.n[2];
    P.N = p.N;
    P.s1_comp = (long)p.n[2] * p.n[1] * p.Hxp;
    P.Hxp = p.Hxp;
    P.with_demag = (terms & MM_DEMAG) ? 1 : 0;
    P.with_exch = (terms & MM_EXCH) && (p.A != 0.0 || p.percell_A) ? 1 : 0;
    P.with_dmi = (terms & MM_DMI) && p.dmi ? 1 : 0;
    // stencil variant (EXT_* bits); a per-cell constant moves into the
    // neighbour-pair average, leaving 2 / mu0 as the prefactor
    int ext = (P.with_dmi ? EXT_DMI : 0) | (P.with_exch && p.percell_A ? EXT_PA : 0) |
              (P.with_dmi && p.percell_D ? EXT_PD : 0) |
              (P.with_dmi && p.percell_D && p.dmi_mixed ? EXT_MIX : 0);
    if (ext == 0 && (terms & MM_ANIS) && p.percell_Ku) ext = EXT_PK;
    P.dmi = 2.0 * ((ext & EXT_PD) ? 1.0 : p.D) / kMu0;
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a)
            P.edmi[k][a] = p.edmi[k][a] / (k == 2 && p.layered ? 1.0 : 2.0 * p.d[k]);
    P.with_anis_hi = p.Ku2 != 0.0 || p.Kc1 != 0.0 || p.Kc2 != 0.0 ? 1 : 0;
    P.with_anis = (terms & MM_ANIS) && (p.Ku != 0.0 || P.with_anis_hi || p.percell_Ku) ? 1 : 0;
    P.with_zee = (terms & MM_ZEEMAN) ? 1 : 0;
    P.with_oe = (terms & MM_OERSTED) && p.oe_on ? 1 : 0;
    P.oe_scale = p.oe_freq != 0.0 ? sin(2.0 * M_PI * p.oe_freq * t) : 1.0;
    P.anis2 = 4.0 * p.Ku2 / kMu0;
    P.cub1 = 2.0 * p.Kc1 / kMu0;
    P.cub2 = 2.0 * p.Kc2 / kMu0;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) P.ec[i][a] = p.ec[i][a];
    P.Ms = p.Ms;
    P.exch = 2.0 * ((ext & EXT_PA) ? 1.0 : p.A) / kMu0;
    P.idx2 = 1.0 / (p.d[0] * p.d[0]);
    P.idy2 = 1.0 / (p.d[1] * p.d[1]);
    P.idz2 = 1.0 / (p.d[2] * p.d[2]);
    P.anis = 2.0 * (p.percell_Ku ? 1.0 : p.Ku) / kMu0;
    for (int a = 0; a < 3; ++a) {
        P.eu[a] = p.eu[a];
        P.H[a] = hext ? hext[a] : 0.0;
        P.Hd[a] = 0.0;
    }
    if (p.drive && p.mask) {
        const double s = sin(2.0 * M_PI * p.drive_freq * t);
        for (int a = 0; a < 3; ++a) P.Hd[a] = p.drive_amp[a] * s;
    }
    P.gp = kGamma / (1.0 + alpha_eff * alpha_eff);
    P.alpha = alpha_eff;
    P.precess = precess ? 1 : 0;
    *ext_out = ext;
    return P;
}

size_t batch_slot_bytes() { return sizeof(LocalParams) + sizeof(double); }

hipError_t batch_init_slots(Plan& g)
{
    if (g.batch <= 1 || !g.Pb || !g.Ms_b || !g.Pb_host) return hipErrorInvalidValue;
    // the plan's geometry, no material: an empty slot's field and right-hand
    // side are zero
    int ext = 0;
    LocalParams P = make_local_params(g, nullptr, 0u, 0.0, 1.0, false, &ext);
    P.Ms = 0.0;
    char* stage = static_cast<char*>(g.Pb_host);
    LocalParams* hp = reinterpret_cast<LocalParams*>(stage);
    for (int b = 0; b < g.batch; ++b) hp[b] = P;
    double* hm = reinterpret_cast<double*>(stage + sizeof(LocalParams) * g.batch);
    std::memset(hm, 0, sizeof(double) * g.batch);
    hipError_t e = hipMemcpyAsync(g.Pb, hp, sizeof(LocalParams) * g.batch, hipMemcpyHostToDevice,
                                  g.stream);
    if (e != hipSuccess) return e;
    const size_t es = g.prec == MM_FP32 ? sizeof(float) : sizeof(double);
    return hipMemcpyAsync(g.Ms_b, hm, es * g.batch, hipMemcpyHostToDevice, g.stream);
}

// Batches run the wave-local z pass and local pass only.
template <typename T>
static bool batch_kernels_ok(int L, int M)
{
    bool mid = false, loc = false;
    switch (L) {
#define MMX_B(LL) \
    case LL: mid = MMX_MIDW && MidW<T, LL>::kOK; break;
        MMX_CASES(MMX_B)
#undef MMX_B
    }
    switch (M) {
#define MMX_B(LL) \
    case LL: loc = MMX_X1W && XC2RW<T, LL>::kOK; break;
        MMX_CASES(MMX_B)
#undef MMX_B
    }
    return mid && loc;
}

template <typename T>
static bool local_wave_ok(int M)
{
    switch (M) {
#define MMX_B(LL) \
    case LL: return MMX_X1W && XC2RW<T, LL>::kOK;
        MMX_CASES(MMX_B)
#undef MMX_B
    }
    return false;
}

bool split_state_ok(const Plan& p, unsigned terms)
{
    if (p.prec != MM_FP32 || p.Pb || p.batch != 1 || p.percell || p.layered) return false;
    // static fields: no drive, no oscillating current
    if (p.drive && p.mask) return false;
    if ((terms & MM_OERSTED) && p.oe_on && p.oe_freq != 0.0) return false;
    int ext = 0;
    (void)make_local_params(p, nullptr, terms, 0.0, 1.0, false, &ext);
    return ext == 0 && local_wave_ok<float>(p.P[0] / 2);
}

bool err_fusable(const Plan& p, unsigned terms)
{
    if (!(terms & MM_DEMAG) || p.P[0] / 2 < 2 || p.Pb || !p.epart || p.batch != 1)
        return false;
    int ext = 0;
    (void)make_local_params(p, nullptr, terms, 0.0, 1.0, true, &ext);
    if (ext != 0) return false;
    const int M = p.P[0] / 2;
    return p.prec == MM_FP32 ? local_wave_ok<float>(M) : local_wave_ok<double>(M);
}

bool batch_supported(const int grid[3], int prec)
{
    int P[3];
    for (int a = 0; a < 3; ++a) P[a] = padded_extent(grid[a]);
    const int M = P[0] / 2, L = P[2] > 1 ? P[2] : P[1];
    if (M < 2) return false;
    return prec == MM_FP32 ? batch_kernels_ok<float>(L, M) : batch_kernels_ok<double>(L, M);
}

hipError_t batch_set_slot(Plan& g, int b, const Plan& v, const double hext[3], unsigned terms,
                          double alpha_eff, bool precess)
{
    if (g.batch <= 1 || b < 0 || b >= g.batch || !g.Pb || !g.Ms_b || !g.Pb_host)
        return hipErrorInvalidValue;
    int ext = 0;
    const LocalParams P = make_local_params(v, hext, terms, 0.0, alpha_eff, precess, &ext);
    if (ext != 0 || v.percell) return hipErrorInvalidValue;
    // staging entry b: its LocalParams, then (after all of them) its Ms
    char* stage = static_cast<char*>(g.Pb_host);
    LocalParams* hp = reinterpret_cast<LocalParams*>(stage) + b;
    double* hm = reinterpret_cast<double*>(stage + sizeof(LocalParams) * g.batch) + b;
    *hp = P;
    size_t ms_bytes;
    if (g.prec == MM_FP32) {
        const float f = (float)v.Ms;
        std::memcpy(hm, &f, sizeof f);
        ms_bytes = sizeof f;
    } else {
        *hm = v.Ms;
        ms_bytes = sizeof(double);
    }
    hipError_t e = hipMemcpyAsync(static_cast<LocalParams*>(g.Pb) + b, hp, sizeof(LocalParams),
                                  hipMemcpyHostToDevice, g.stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(static_cast<char*>(g.Ms_b) + (size_t)b * ms_bytes, hm, ms_bytes,
                          hipMemcpyHostToDevice, g.stream);
}

// sc: the x forward pass forms the stage input sc (m == sc->ys) from its
// parts instead of reading m.  err (with sc->ep): the local pass also
// accumulates the error norm into err->out_dev.
template <typename T>
static hipError_t eval_field_core(Plan& p, const T* m, const double hext[3], unsigned terms,
                                  double t, T* h_out, T* dm_out, double alpha_eff, bool precess,
                                  double* torque, const StageIn<T>* sc,
                                  const ErrIn<T>* err = nullptr, const T* m_lo = nullptr)
{
    const int M = p.P[0] / 2;
    const bool pc = p.percell;
    // a batch plan (p.Pb; p.batch of its requests per launch): uniform
    // material and the plain stencil only, at most 64 requests
    if (p.Pb && (pc || p.percell_A || p.percell_D || p.percell_Ku || p.dmi || p.layered ||
                 p.batch > 64 || !p.Ms_b))
        return hipErrorInvalidValue;
    if (!p.Pb && p.batch != 1) return hipErrorInvalidValue;
    if (terms & MM_DEMAG) MMX_TRY(demag_to_S1<T>(p, sc ? sc->y : m, true, sc));
    int ext = 0;
    const LocalParams P = make_local_params(p, hext, terms, t, alpha_eff, precess, &ext);
    if (torque) {
        // a batch keeps one maximum per request, 8 doubles apart
        if (p.Pb)
            k_fill_strided<<<1, 64, 0, p.stream>>>(torque, p.batch, 8, 0.0);
        else
            k_fill<<<1, 64, 0, p.stream>>>(torque, 1, 0.0);
        MMX_TRY(hipGetLastError());
    }
    if (err) {
        // the error norm accumulated by the local pass: block partials, then
        // the final sums as in rk_error_norm
        if (ext != 0 || !sc || !sc->ep || !p.epart) return hipErrorInvalidValue;
        const LocalErr<T> le{sc->ep, err->y, err->e6, err->rtol, err->atol, p.epart};
        long nb = 0;
        MMX_TRY(timed(p, MM_PASS_X_INV_LOCAL, [&] {
            return pc ? launch_local<T, true, 0>(p, M, m, h_out, dm_out, P, torque, &le, &nb)
                      : launch_local<T, false, 0>(p, M, m, h_out, dm_out, P, torque, &le, &nb);
        }));
        const double cnt = 3.0 * (double)p.n_magnetic;
        k_err_sums<<<1, kSumBlock, 0, p.stream>>>(p.epart, (int)nb, 2 * nb, err->out_dev, 8,
                                                  cnt > 0 ? 1.0 / cnt : 0.0, nullptr);
        return hipGetLastError();
    }
    // DMI and the coupling averages only in the variants that need them.
    // The split state needs the wave-local pass; elsewhere the float part
    // alone is used
    if (m_lo && (ext != 0 || pc || sc)) return hipErrorInvalidValue;
    if (m_lo && !(std::is_same<T, float>::value && local_wave_ok<T>(M))) m_lo = nullptr;
    return timed(p, MM_PASS_X_INV_LOCAL, [&] {
        if (ext == 0)
            return pc ? launch_local<T, true, 0>(p, M, m, h_out, dm_out, P, torque)
                      : launch_local<T, false, 0>(p, M, m, h_out, dm_out, P, torque, nullptr,
                                                  nullptr, m_lo);
        return launch_local_ext<T>(p, M, m, h_out, dm_out, P, torque, pc, ext);
    });
}

template <typename T>
hipError_t eval_field(Plan& p, const T* m, const double hext[3], unsigned terms, double t,
                      T* h_out, T* dm_out, double alpha_eff, bool precess, double* torque,
                      const T* m_lo)
{
    return eval_field_core<T>(p, m, hext, terms, t, h_out, dm_out, alpha_eff, precess, torque,
                              nullptr, nullptr, m_lo);
}

template <typename T>
hipError_t eval_field_stage(Plan& p, const StageIn<T>& sc, const double hext[3], unsigned terms,
                            double t, T* dm_out, double alpha_eff, bool precess, double* torque,
                            const ErrIn<T>* err)
{
    if (sc.nk < 1 || sc.nk > 7 || !sc.y || !sc.ys) return hipErrorInvalidValue;
    if (err || sc.ep) {
        if (!(err && sc.ep) || !err_fusable(p, terms)) return hipErrorInvalidValue;
        return eval_field_core<T>(p, sc.ys, hext, terms, t, nullptr, dm_out, alpha_eff, precess,
                                  torque, &sc, err);
    }
    // a batch forms its stage inputs in the combination kernel (one step
    // size per request)
    if (!(terms & MM_DEMAG) || p.P[0] / 2 < 2 || p.Pb) {
        MMX_TRY(rk_combine<T>(p, sc.ys, sc.y, 1.0, sc.c, const_cast<T* const*>(sc.k), sc.nk,
                              sc.h));
        return eval_field_core<T>(p, sc.ys, hext, terms, t, nullptr, dm_out, alpha_eff, precess,
                                  torque, nullptr);
    }
    return eval_field_core<T>(p, sc.ys, hext, terms, t, nullptr, dm_out, alpha_eff, precess,
                              torque, &sc);
}

// ---------------------------------------------------------------------------
// Runge-Kutta helpers.
// ---------------------------------------------------------------------------
static bool aligned16(const void* q) { return ((uintptr_t)q & 15) == 0; }

// The error norm's final sums from its nb (sum, non-finite count) partial
// pairs: out_dev[0] = RMS over the magnetic components, out_dev[5] = number
// of non-finite entries of the current state; per request of a batch (its
// partials 2 nb apart, its results 8 doubles apart); with ctl, the same
// launch then takes each request's step decision.
static hipError_t err_final_sums(Plan& p, int nb, double* out_dev, DevCtl* ctl = nullptr)
{
    const double cnt = 3.0 * (double)p.n_magnetic;
    const double sc = cnt > 0 ? 1.0 / cnt : 0.0;
    k_err_sums<<<std::max(1, p.batch), kSumBlock, 0, p.stream>>>(p.red, nb, 2L * nb, out_dev, 8,
                                                                 sc, ctl);
    return hipGetLastError();
}

template <typename T, int NK>
static hipError_t launch_combine(Plan& p, T* y_out, const T* y, const Coef7& cf, const Ptr7<T>& ks,
                                 bool vec)
{
    const long n3 = 3 * p.N;
    const long work = vec ? n3 / V16<T>::n : n3;
    const dim3 grid((unsigned)std::min<long>(blocks_for(work, 256), 8192), (unsigned)p.batch);
    if (vec)
        k_rk_combine<T, NK, true><<<grid, 256, 0, p.stream>>>(y_out, y, cf, ks, n3);
    else
        k_rk_combine<T, NK, false><<<grid, 256, 0, p.stream>>>(y_out, y, cf, ks, n3);
    return hipGetLastError();
}

template <typename T>
hipError_t rk_combine(Plan& p, T* y_out, const T* y, double h, const double* a, T* const* k, int nk,
                      const double* hdev)
{
    Coef7 cf{};
    Ptr7<T> ks{};
    cf.h = hdev;
    cf.hstride = hdev && p.batch > 1 ? kCtlStride : 0;
    bool vec = (p.N % V16<T>::n) == 0 && aligned16(y_out) && aligned16(y);
    for (int j = 0; j < nk; ++j) {
        cf.c[j] = hdev ? a[j] : h * a[j];
        ks.p[j] = k[j];
        vec = vec && aligned16(k[j]);
    }
    return timed(p, MM_PASS_RK, [&] {
        switch (nk) {
        case 1: return launch_combine<T, 1>(p, y_out, y, cf, ks, vec);
        case 2: return launch_combine<T, 2>(p, y_out, y, cf, ks, vec);
        case 3: return launch_combine<T, 3>(p, y_out, y, cf, ks, vec);
        case 4: return launch_combine<T, 4>(p, y_out, y, cf, ks, vec);
        case 5: return launch_combine<T, 5>(p, y_out, y, cf, ks, vec);
        case 6: return launch_combine<T, 6>(p, y_out, y, cf, ks, vec);
        case 7: return launch_combine<T, 7>(p, y_out, y, cf, ks, vec);
        }
        return hipErrorInvalidValue;
    });
}

template <typename T>
hipError_t rk_error_norm(Plan& p, const T* y, const T* y1, double h, const double* e, T* const* k,
                         int nk, double rtol, double atol, double* out_dev, const double* hdev,
                         DevCtl* ctl)
{
    Coef7 cf{};
    Ptr7<T> ks{};
    cf.h = hdev;
    cf.hstride = hdev && p.batch > 1 ? kCtlStride : 0;
    bool vec = (p.N % V16<T>::n) == 0 && aligned16(y) && aligned16(y1) &&
               (!p.percell || aligned16(p.Ms_cell));
    for (int j = 0; j < 7; ++j) {
        cf.c[j] = j < nk ? (hdev ? e[j] : h * e[j]) : 0.0;
        ks.p[j] = j < nk ? k[j] : y;
        vec = vec && aligned16(ks.p[j]);
    }
    const T* msc = p.percell ? (const T*)p.Ms_cell : nullptr;
    // a streaming reduction: about 4 (vector) elements per thread, up to
    // kErrBlocks blocks, so large grids keep 8 waves per SIMD resident and
    // mid-sized ones (the served grids) still fill the chip (partials: sums
    // in [0, nb), non-finite counts in [nb, 2 nb)); nb depends on the grid only
    const long nv = 3 * p.N / (vec ? V16<T>::n : 1);
    const int nb = (int)std::max<long>(1, std::min<long>(kErrBlocks, blocks_for(nv, kBlock * 4)));
    if (p.batch > 1 && p.percell) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb, (unsigned)p.batch);
    MMX_TRY(timed(p, MM_PASS_RK, [&] {
        if (vec && p.percell)
            k_err_norm<T, true, true><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol,
                                                                     atol, p.red);
        else if (vec)
            k_err_norm<T, true, false><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc,
                                                                      rtol, atol, p.red);
        else if (p.percell)
            k_err_norm<T, false, true><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc,
                                                                      rtol, atol, p.red);
        else
            k_err_norm<T, false, false><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc,
                                                                       rtol, atol, p.red);
        return hipGetLastError();
    }));
    return err_final_sums(p, nb, out_dev, ctl);
}

template <typename T>
hipError_t renormalise(Plan& p, T* m)
{
    const int blocks = (int)std::min<long>(blocks_for(p.N, 256), 4096);
    k_renorm<T><<<blocks, 256, 0, p.stream>>>(m, p.percell ? (const T*)p.Ms_cell : nullptr, p.N);
    return hipGetLastError();
}

// One controller thread per request (a batch's controllers are adjacent, its
// reduction results 8 doubles apart).
hipError_t dp_begin(Plan& p, DevCtl* c)
{
    k_dp_begin<<<1, p.batch, 0, p.stream>>>(c, p.red_out, p.batch, 8);
    return hipGetLastError();
}

hipError_t dp_torque(Plan& p, DevCtl* c)
{
    k_dp_torque<<<1, p.batch, 0, p.stream>>>(c, p.red_out, p.batch, 8);
    return hipGetLastError();
}

template <typename T>
hipError_t dp_commit(Plan& p, DevCtl* c, T* y, const T* y1, T* k0, const T* k6)
{
    if (p.batch > 1 && p.percell) return hipErrorInvalidValue;
    const dim3 grid((unsigned)std::min<long>(blocks_for(p.N, 256), 4096), (unsigned)p.batch);
    k_dp_commit<T><<<grid, 256, 0, p.stream>>>(c, y, y1, k0, k6,
                                               p.percell ? (const T*)p.Ms_cell : nullptr, p.N);
    return hipGetLastError();
}

template <typename T>
hipError_t anis_energy(Plan& p, const T* m, double* out_dev, double* partials)
{
    double* red = partials ? partials : p.red;
    AnisE A;
    A.ku1 = p.Ku;
    A.ku2 = p.Ku2;
    A.kc1 = p.Kc1;
    A.kc2 = p.Kc2;
    for (int a = 0; a < 3; ++a) {
        A.eu[a] = p.eu[a];
        for (int b = 0; b < 3; ++b) A.ec[a][b] = p.ec[a][b];
    }
    k_anis_energy<T><<<kRedBlocks, kBlock, 0, p.stream>>>(
        m, p.percell ? (const T*)p.Ms_cell : nullptr, p.Ms, p.N, A, red,
        p.layered ? p.lw : nullptr, (long)p.n[0] * p.n[1],
        p.percell_Ku ? (const T*)p.Ku_cell : nullptr);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(red, kRedBlocks, out_dev, 0, 1.0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t dot_ms(Plan& p, const T* a, const T* b, double* out_dev, double* partials)
{
    double* red = partials ? partials : p.red;
    k_dot_ms<T><<<kRedBlocks, kBlock, 0, p.stream>>>(a, b, p.percell ? (const T*)p.Ms_cell : nullptr,
                                                     p.Ms, p.N, red, p.layered ? p.lw : nullptr,
                                                     (long)p.n[0] * p.n[1]);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(red, kRedBlocks, out_dev, 0, 1.0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t start_norms(Plan& p, const T* y, const T* f0, const T* f1, double rtol, double atol,
                       double* out_dev)
{
    k_start_norms<T><<<kRedBlocks, kBlock, 0, p.stream>>>(
        y, f0, f1, p.percell ? (const T*)p.Ms_cell : nullptr, p.N, rtol, atol, p.red);
    MMX_TRY(hipGetLastError());
    for (int i = 0; i < 3; ++i) {
        k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red + i * kRedBlocks, kRedBlocks, out_dev, i, 1.0,
                                                0);
        MMX_TRY(hipGetLastError());
    }
    return hipSuccess;
}

template <typename T>
hipError_t count_magnetic(Plan& p, double* out_dev)
{
    k_count_mag<T><<<kRedBlocks, kBlock, 0, p.stream>>>((const T*)p.Ms_cell, p.N, p.red);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red, kRedBlocks, out_dev, 0, 1.0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t count_signs(Plan& p, const T* v, double* out_dev)
{
    k_count_signs<T><<<kRedBlocks, kBlock, 0, p.stream>>>(v, p.N, p.red);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red, kRedBlocks, out_dev, 0, 1.0, 0);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red + kRedBlocks, kRedBlocks, out_dev, 1, 1.0, 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Differentiation host pipeline.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t field_vjp(Plan& p, const T* m, const T* w, const T* h, unsigned terms, double alpha,
                     T* g_tmp, T* z_tmp, T* nu, double* gms)
{
    const int blocks = (int)std::min<long>(blocks_for(p.N, 256), 4096);
    const double gp = kGamma / (1.0 + alpha * alpha);
    if (p.percell)
        k_vjp_pre<T, true><<<blocks, 256, 0, p.stream>>>(m, h, w, (const T*)p.Ms_cell, (T)p.Ms, p.N,
                                                       (T)gp, (T)alpha, h ? g_tmp : nullptr,
                                                       z_tmp);
    else
        k_vjp_pre<T, false><<<blocks, 256, 0, p.stream>>>(m, h, w, nullptr, (T)p.Ms, p.N, (T)gp,
                                                        (T)alpha, h ? g_tmp : nullptr, z_tmp);
    MMX_TRY(hipGetLastError());
    const bool demag = (terms & MM_DEMAG) != 0;
    if (demag) MMX_TRY(demag_to_S1<T>(p, z_tmp, false));
    AdjParams P;
    P.nx = p.n[0];
    P.ny = p.n[1];
    P.nz = p.n[2];
    P.N = p.N;
    P.s1_comp = (long)p.n[2] * p.n[1] * p.Hxp;
    P.Hxp = p.Hxp;
    P.with_demag = demag ? 1 : 0;
    P.with_exch = (terms & MM_EXCH) && p.A != 0.0 ? 1 : 0;
    P.with_anis = (terms & MM_ANIS) && p.Ku != 0.0 ? 1 : 0;
    P.Ms = p.Ms;
    P.exch = 2.0 * p.A / kMu0;
    P.idx2 = 1.0 / (p.d[0] * p.d[0]);
    P.idy2 = 1.0 / (p.d[1] * p.d[1]);
    P.idz2 = 1.0 / (p.d[2] * p.d[2]);
    P.anis = 2.0 * p.Ku / kMu0;
    for (int a = 0; a < 3; ++a) P.eu[a] = p.eu[a];
    const int M = p.P[0] / 2;
    const T* g = h ? g_tmp : nullptr;
    return timed(p, MM_PASS_X_INV_LOCAL, [&] {
        return p.percell ? launch_adj<T, true>(p, M, m, z_tmp, g, nu, gms, P)
                         : launch_adj<T, false>(p, M, m, z_tmp, g, nu, gms, P);
    });
}

template <typename T>
hipError_t lincomb(Plan& p, T* out, const double* c, T* const* v, int nk)
{
    Coef7 cf{};
    Ptr7<T> ps{};
    for (int j = 0; j < nk; ++j) {
        cf.c[j] = c[j];
        ps.p[j] = v[j];
    }
    const long n3 = 3 * p.N;
    const int blocks = (int)std::min<long>(blocks_for(n3, 256), 8192);
    return timed(p, MM_PASS_RK, [&] {
        switch (nk) {
        case 1: k_lincomb<T, 1><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        case 2: k_lincomb<T, 2><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        case 3: k_lincomb<T, 3><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        case 4: k_lincomb<T, 4><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        case 5: k_lincomb<T, 5><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        case 6: k_lincomb<T, 6><<<blocks, 256, 0, p.stream>>>(out, cf, ps, n3); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
}

template <typename T>
hipError_t region_mz_accum(Plan& p, const T* m, const unsigned char* region, double* out_dev,
                           double scale)
{
    k_region_mz<T><<<kRedBlocks, kBlock, 0, p.stream>>>(m, region, p.N, p.red);
    MMX_TRY(hipGetLastError());
    k_final_accum<<<1, kBlock, 0, p.stream>>>(p.red, kRedBlocks, out_dev, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t add_region(Plan& p, T* lam, const unsigned char* region, double val)
{
    const int blocks = (int)std::min<long>(blocks_for(p.N, 256), 4096);
    k_add_region<T><<<blocks, 256, 0, p.stream>>>(lam, region, p.N, (T)val);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Double state with single-precision stages (relaxations and served requests
// of FP32 plans, Plan::state64): the Runge-Kutta state y and trial state y1
// are kept in double, the stage derivatives k_j are the FP32 pipeline's
// outputs, and each stage input is formed in double and rounded once to float
// for the field evaluation.  An FP32 state would be rounded by ~6e-8 per
// component every step, a perturbation as large as the tolerances the
// relaxation criterion needs, which the exchange stencil turns into torque.
// ---------------------------------------------------------------------------
template <int NK>
__global__ __launch_bounds__(kBlock) void k_rk_combine_d(float* __restrict__ ys,
                                                         double* __restrict__ y1,
                                                         const double* __restrict__ y, Coef7 cf,
                                                         Ptr7<float> ks, long n3,
                                                         float* __restrict__ ys_lo)
{
    // request blockIdx.y of a batch
    const long bo = (long)blockIdx.y * n3;
    ys += bo;
    if (y1) y1 += bo;
    if (ys_lo) ys_lo += bo;
    y += bo;
#pragma unroll
    for (int j = 0; j < NK; ++j) ks.p[j] += bo;
    const double hs = cf.h ? cf.h[blockIdx.y * cf.hstride] : 1.0;
    double cj[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) cj[j] = cf.c[j] * hs;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n3;
         q += (long)gridDim.x * blockDim.x) {
        double acc = y[q];
#pragma unroll
        for (int j = 0; j < NK; ++j)
            if (cf.c[j] != 0.0) acc += cj[j] * (double)ks.p[j][q];
        if (y1) y1[q] = acc;
        const float hi = (float)acc;
        ys[q] = hi;
        if (ys_lo) ys_lo[q] = (float)(acc - (double)hi);
    }
}

// Sum over magnetic components of (e/sc)^2, e = sum_j c_j k_j, sc = atol +
// rtol max(|y|, |y1|), with y, y1 in double; non-finite entries of y counted.
template <bool PERCELL>
__global__ __launch_bounds__(kBlock) void k_err_norm_d(const double* __restrict__ y,
                                                       const double* __restrict__ y1, Coef7 cf,
                                                       Ptr7<float> ks, long N,
                                                       const float* __restrict__ Ms_cell,
                                                       double rtol, double atol, double* partials)
{
    // request blockIdx.y of a batch (uniform material)
    const long bo = (long)blockIdx.y * 3 * N;
    y += bo;
    y1 += bo;
#pragma unroll
    for (int j = 0; j < 7; ++j) ks.p[j] += bo;
    partials += (long)blockIdx.y * 2 * gridDim.x;
    const double hs = cf.h ? cf.h[blockIdx.y * cf.hstride] : 1.0;
    double cj[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) cj[j] = cf.c[j] * hs;
    double acc = 0.0, bad = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < 3 * N;
         q += (long)gridDim.x * blockDim.x) {
        const double a = y[q], b = y1[q];
        if (!isfinite(a)) bad += 1.0;
        if (PERCELL && Ms_cell[q % N] == 0.0f) continue;
        double e = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (cf.c[j] != 0.0) e += cj[j] * (double)ks.p[j][q];
        const double sc = atol + rtol * fmax(fabs(a), fabs(b));
        const double r = e / sc;
        acc += r * r;
    }
    acc = block_sum(acc);
    bad = block_sum(bad);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = acc;
        partials[gridDim.x + blockIdx.x] = bad;
    }
}

// On acceptance: y = y1 (renormalised on magnetic cells, zero on vacuum, when
// c->renorm) with its float copy ys; without renorm k0 = k6 (first-same-as-
// last: ys already holds the rounded y1 the last stage was evaluated at).
// With renorm the step ends by evaluating k0 at ys, so on a rejection ys is
// reset to the rounded, unchanged y (it held the rejected trial state).
__global__ void k_dp_commit_d(const DevCtl* __restrict__ c, double* __restrict__ y,
                              const double* __restrict__ y1, float* __restrict__ ys,
                              float* __restrict__ k0, const float* __restrict__ k6,
                              const float* __restrict__ Ms_cell, long N, float* __restrict__ ys_lo)
{
    // request blockIdx.y of a batch
    const long bo = (long)blockIdx.y * 3 * N;
    c += blockIdx.y;
    y += bo;
    y1 += bo;
    ys += bo;
    if (ys_lo) ys_lo += bo;
    k0 += bo;
    k6 += bo;
    const bool commit = c->commit != 0;
    const bool renorm = c->renorm != 0;
    if (!commit && !renorm) return;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
         q += (long)gridDim.x * blockDim.x) {
        if (!commit) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double v = y[a * N + q];
                const float hi = (float)v;
                ys[a * N + q] = hi;
                if (ys_lo) ys_lo[a * N + q] = (float)(v - (double)hi);
            }
            continue;
        }
        double x = y1[q], yy = y1[N + q], z = y1[2 * N + q];
        if (renorm) {
            if (Ms_cell && Ms_cell[q] == 0.0f) {
                x = yy = z = 0.0;
            } else {
                const double inv = 1.0 / sqrt(x * x + yy * yy + z * z);
                x *= inv;
                yy *= inv;
                z *= inv;
            }
            const float hx = (float)x, hy = (float)yy, hz = (float)z;
            ys[q] = hx;
            ys[N + q] = hy;
            ys[2 * N + q] = hz;
            if (ys_lo) {
                ys_lo[q] = (float)(x - (double)hx);
                ys_lo[N + q] = (float)(yy - (double)hy);
                ys_lo[2 * N + q] = (float)(z - (double)hz);
            }
        } else {
            k0[q] = k6[q];
            k0[N + q] = k6[N + q];
            k0[2 * N + q] = k6[2 * N + q];
        }
        y[q] = x;
        y[N + q] = yy;
        y[2 * N + q] = z;
    }
}

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ in, B* __restrict__ out, long n)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        out[q] = (B)in[q];
}

hipError_t rk_combine_d(Plan& p, float* ys, double* y1, const double* y, const double* a,
                        float* const* k, int nk, const double* hdev, float* ys_lo)
{
    Coef7 cf{};
    Ptr7<float> ks{};
    cf.h = hdev;
    cf.hstride = hdev && p.batch > 1 ? kCtlStride : 0;
    for (int j = 0; j < nk; ++j) {
        cf.c[j] = a[j];
        ks.p[j] = k[j];
    }
    const long n3 = 3 * p.N;
    const dim3 blocks((unsigned)std::min<long>(blocks_for(n3, kBlock), 8192), (unsigned)p.batch);
    return timed(p, MM_PASS_RK, [&] {
        switch (nk) {
#define MMX_CD(NK) \
    case NK:                                                                                 \
        k_rk_combine_d<NK><<<blocks, kBlock, 0, p.stream>>>(ys, y1, y, cf, ks, n3, ys_lo);     \
        break;
            MMX_CD(1) MMX_CD(2) MMX_CD(3) MMX_CD(4) MMX_CD(5) MMX_CD(6) MMX_CD(7)
#undef MMX_CD
        default:
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
}

hipError_t rk_error_norm_d(Plan& p, const double* y, const double* y1, const double* e,
                           float* const* k, int nk, double rtol, double atol, double* out_dev,
                           const double* hdev, DevCtl* ctl)
{
    Coef7 cf{};
    Ptr7<float> ks{};
    cf.h = hdev;
    cf.hstride = hdev && p.batch > 1 ? kCtlStride : 0;
    for (int j = 0; j < 7; ++j) {
        cf.c[j] = j < nk ? e[j] : 0.0;
        ks.p[j] = j < nk ? k[j] : k[0];
    }
    const float* msc = p.percell ? (const float*)p.Ms_cell : nullptr;
    if (p.batch > 1 && msc) return hipErrorInvalidValue;
    const int nb = (int)std::max<long>(1, std::min<long>(kErrBlocks, blocks_for(3 * p.N, kBlock * 4)));
    const dim3 grid((unsigned)nb, (unsigned)p.batch);
    MMX_TRY(timed(p, MM_PASS_RK, [&] {
        if (msc)
            k_err_norm_d<true><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol, atol,
                                                              p.red);
        else
            k_err_norm_d<false><<<grid, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol, atol,
                                                               p.red);
        return hipGetLastError();
    }));
    return err_final_sums(p, nb, out_dev, ctl);
}

hipError_t dp_commit_d(Plan& p, DevCtl* c, double* y, const double* y1, float* ys, float* k0,
                       const float* k6, float* ys_lo)
{
    if (p.batch > 1 && p.percell) return hipErrorInvalidValue;
    const dim3 blocks((unsigned)std::min<long>(blocks_for(p.N, 256), 4096), (unsigned)p.batch);
    k_dp_commit_d<<<blocks, 256, 0, p.stream>>>(c, y, y1, ys, k0, k6,
                                                p.percell ? (const float*)p.Ms_cell : nullptr, p.N,
                                                ys_lo);
    return hipGetLastError();
}

hipError_t convert_f32_f64(Plan& p, const float* in, double* out, long n)
{
    const int blocks = (int)std::min<long>(blocks_for(n, 256), 4096);
    k_convert<float, double><<<blocks, 256, 0, p.stream>>>(in, out, n);
    return hipGetLastError();
}

hipError_t convert_f64_f32(Plan& p, const double* in, float* out, long n)
{
    const int blocks = (int)std::min<long>(blocks_for(n, 256), 4096);
    k_convert<double, float><<<blocks, 256, 0, p.stream>>>(in, out, n);
    return hipGetLastError();
}

hipError_t zero_doubles(Plan& p, double* ptr, long n)
{
    const int blocks = (int)std::min<long>(blocks_for(n, 256), 4096);
    k_zero_d<<<blocks, 256, 0, p.stream>>>(ptr, n);
    return hipGetLastError();
}

template <typename T>
hipError_t from_double(Plan& p, const double* in, T* out, long n)
{
    const int blocks = (int)std::min<long>(blocks_for(n, 256), 4096);
    k_from_double<T><<<blocks, 256, 0, p.stream>>>(in, out, n);
    return hipGetLastError();
}

#define MMX_INST(T)                                                                              \
    template hipError_t build_tensor<T>(Plan&);                                                  \
    template hipError_t init_twiddles<T>(Plan&);                                                 \
    template hipError_t eval_field<T>(Plan&, const T*, const double*, unsigned, double, T*, T*, \
                                      double, bool, double*, const T*);                          \
    template hipError_t eval_field_stage<T>(Plan&, const StageIn<T>&, const double*, unsigned,   \
                                            double, T*, double, bool, double*,                   \
                                            const ErrIn<T>*);                                    \
    template hipError_t rk_combine<T>(Plan&, T*, const T*, double, const double*, T* const*,     \
                                      int, const double*);                                       \
    template hipError_t rk_error_norm<T>(Plan&, const T*, const T*, double, const double*,       \
                                         T* const*, int, double, double, double*, const double*,  \
                                         DevCtl*);                                                \
    template hipError_t dp_commit<T>(Plan&, DevCtl*, T*, const T*, T*, const T*);                \
    template hipError_t renormalise<T>(Plan&, T*);                                               \
    template hipError_t dot_ms<T>(Plan&, const T*, const T*, double*, double*);                  \
    template hipError_t anis_energy<T>(Plan&, const T*, double*, double*);                       \
    template hipError_t start_norms<T>(Plan&, const T*, const T*, const T*, double, double,      \
                                       double*);                                                 \
    template hipError_t count_magnetic<T>(Plan&, double*);                                       \
    template hipError_t count_signs<T>(Plan&, const T*, double*);                                \
    template hipError_t oersted_field<T>(Plan&, const T*, T*);                                   \
    template hipError_t debug_spectrum<T>(Plan&, int, double*);                                  \
    template hipError_t field_vjp<T>(Plan&, const T*, const T*, const T*, unsigned, double, T*,  \
                                     T*, T*, double*);                                           \
    template hipError_t lincomb<T>(Plan&, T*, const double*, T* const*, int);                    \
    template hipError_t region_mz_accum<T>(Plan&, const T*, const unsigned char*, double*,       \
                                           double);                                              \
    template hipError_t add_region<T>(Plan&, T*, const unsigned char*, double);                  \
    template hipError_t from_double<T>(Plan&, const double*, T*, long);

MMX_INST(float)
MMX_INST(double)

}  // namespace mmx
