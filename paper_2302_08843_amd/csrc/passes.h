// passes.h -- the field passes of the effective-field pipeline (F1 x forward,
// F2/I2 strided y transforms, F3 last-axis transform with the spectral product,
// I1 x inverse with the local terms) and their launchers, shared by the
// translation units that instantiate them.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "engine.h"
#include "fft.h"
#include "newell.h"

namespace mmx {

// Registers per thread in each kind of pass (complex values).  The defaults
// can be overridden at build time for tuning sweeps.
#ifndef MMX_RX_F32
#define MMX_RX_F32 16
#endif
#ifndef MMX_RS_F32
#define MMX_RS_F32 32
#endif
#ifndef MMX_RM_F32
#define MMX_RM_F32 16
#endif
#ifndef MMX_RX1_F32
#define MMX_RX1_F32 8
#endif
#ifndef MMX_RX_F64
#define MMX_RX_F64 16
#endif
#ifndef MMX_RS_F64
#define MMX_RS_F64 16
#endif
#ifndef MMX_RM_F64
#define MMX_RM_F64 8
#endif
#ifndef MMX_RX1_F64
#define MMX_RX1_F64 8
#endif
// threads per block targeted by the strided and last-axis passes
#ifndef MMX_SBLOCK
#define MMX_SBLOCK 512
#endif
#ifndef MMX_MBLOCK
#define MMX_MBLOCK 256
#endif
#ifndef MMX_XBLOCK
#define MMX_XBLOCK 64
#endif
#ifndef MMX_X1BLOCK
#define MMX_X1BLOCK 256
#endif
// z pass: ky and Py - ky in adjacent blocks (ADJ) instead of one after the
// other in one block, so each spectral-kernel row leaves HBM once (measured:
// FP64 faster; FP32 the same time with 26 % less read traffic); block size per
// precision
#ifndef MMX_MBLOCK_F64
#define MMX_MBLOCK_F64 256
#endif
#ifndef MMX_MID_ADJ_F32
#define MMX_MID_ADJ_F32 1
#endif
#ifndef MMX_MID_ADJ_F64
#define MMX_MID_ADJ_F64 1
#endif
// z pass with wave-local transforms (k_mid_w): registers per thread
#ifndef MMX_MIDW
#define MMX_MIDW 1
#endif
#ifndef MMX_RMW_F32
#define MMX_RMW_F32 16
#endif
#ifndef MMX_RMW_F64
#define MMX_RMW_F64 8
#endif
#ifdef MMX_STRIDED_WPE
#define MMX_STRIDED_ATTR __attribute__((amdgpu_waves_per_eu(MMX_STRIDED_WPE)))
#else
#define MMX_STRIDED_ATTR
#endif
// F1 in FP32: 96 VGPRs give 5 waves per SIMD (measured -3 % at 512x512x64)
#ifndef MMX_XR2C_WPE_F32
#define MMX_XR2C_WPE_F32 5
#endif
#define MMX_XR2C_ATTR __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? MMX_XR2C_WPE_F32 : 1)))
#ifdef MMX_MIDW_WPE
#define MMX_MIDW_ATTR __attribute__((amdgpu_waves_per_eu(MMX_MIDW_WPE)))
#else
#define MMX_MIDW_ATTR
#endif
// x inverse / local pass with wave-local transforms and prefetched neighbours
#ifndef MMX_X1W
#define MMX_X1W 1
#endif
#ifndef MMX_SSPLIT
#define MMX_SSPLIT 1  // strided passes: exchange real and imaginary parts separately
#endif
#ifndef MMX_EXT_RCP
#define MMX_EXT_RCP 1  // FP32 harmonic means through the hardware reciprocal
#endif
#ifndef MMX_X1_KFAST
#define MMX_X1_KFAST 1  // x inverse / local pass: consecutive blocks walk z first
#endif
#ifndef MMX_XVEC
#define MMX_XVEC 1  // x forward pass: paired (8 / 16-byte) loads when aligned
#endif
#ifndef MMX_X1BLOCK_F64
#define MMX_X1BLOCK_F64 256
#endif
template <typename T>
struct Regs;
template <>
struct Regs<float> {
    static constexpr int x = MMX_RX_F32;    // F1 row transforms
    static constexpr int s = MMX_RS_F32;    // strided y passes
    static constexpr int mid = MMX_RM_F32;  // F3: three components resident
    static constexpr int x1 = MMX_RX1_F32;  // I1: three components per row
};
template <>
struct Regs<double> {
    static constexpr int x = MMX_RX_F64;
    static constexpr int s = MMX_RS_F64;
    static constexpr int mid = MMX_RM_F64;
    static constexpr int x1 = MMX_RX1_F64;
};

constexpr int kBlock = 256;

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// The dispatcher hands linear workgroup b to XCD (b mod 8), and every XCD has
// its own L2.  Launches below use 1-D grids padded to a multiple of 8 and the
// logical block (b mod 8) * (G/8) + b/8, so each XCD walks one contiguous
// range of logical blocks: neighbouring column tiles that share 128-byte lines
// (and neighbouring rows of the exchange stencil) are then served by the same
// L2 at about the same time.
constexpr int kXCD = 8;
__host__ __device__ inline long xcd_grid(long blocks) { return (blocks + kXCD - 1) / kXCD * kXCD; }
__device__ inline long xcd_logical()
{
    const long G = gridDim.x, b = blockIdx.x;
    return (b % kXCD) * (G / kXCD) + b / kXCD;
}


// ---------------------------------------------------------------------------
// Twiddle table: tw[n] = exp(-2 pi i n / Lmax), rounded from double.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_twiddles(cx<T>* tw, int Lmax)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= Lmax) return;
    double s, c;
    sincospi(-2.0 * (double)n / (double)Lmax, &s, &c);
    tw[n] = {(T)c, (T)s};
}

// ---------------------------------------------------------------------------
// F1: x real-to-complex transform of rows of length 2M (M >= 2).
// Row r of component c reads in[c*in_comp + r*in_row + i] for i < n_in (zero
// beyond) times Ms, and writes X[k], k = 0..M, to out[c*out_comp + r*out_row].
// A real transform of length 2M is a complex transform of length M of
// z[n] = x[2n] + i x[2n+1] followed by the split
//   X[k] = (Z[k] + conj Z[M-k])/2 - i w^k (Z[k] - conj Z[M-k])/2,
//   w = exp(-2 pi i/(2M)).
// ---------------------------------------------------------------------------
// One element of a stage input (StageIn), stored to sc.ys and returned; with
// sc.ep also the partial error sum_j e_j k_j (double, from the same loads).
template <typename T>
__device__ __forceinline__ T stage_elem(const StageIn<T>& sc, const T (&cj)[7],
                                        const double (&ej)[7], long o)
{
    T acc = sc.y[o];
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const bool uc = sc.c[j] != 0.0, ue = sc.ep && sc.e[j] != 0.0;
        if (!uc && !ue) continue;
        const T kv = sc.k[j][o];
        if (uc) acc += cj[j] * kv;
        if (ue) e += ej[j] * (double)kv;
    }
    sc.ys[o] = acc;
    if (sc.ep) sc.ep[o] = (T)e;
    return acc;
}

template <typename T, int M>
struct XR2C {
    using S = FFTShape<M, Regs<T>::x>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kRows = cmax(1, MMX_XBLOCK / kT);
};

// COMB: the rows are those of a Runge-Kutta stage input y + sum_j c_j k_j
// (StageIn; `in` is y), formed here in the order and precision of the
// combination kernel and stored to sc.ys before the Ms scaling.  Ms_b (a
// batch of requests, components 3b..3b+2 of request b): uniform Ms per
// request, Ms_b[c / 3] in place of Ms.
template <typename T, int M, bool PERCELL, bool HALF, bool COMB>
__global__ __launch_bounds__((XR2C<T, M>::kRows * XR2C<T, M>::kT)) MMX_XR2C_ATTR void k_x_r2c(
    const T* __restrict__ in, long in_row, long in_comp, int n_in, const T* __restrict__ Ms_cell,
    T Ms, cx<T>* __restrict__ out, long out_row, long out_comp, int nrows, int ncomp,
    const cx<T>* __restrict__ tw, int Lmax, bool vec, StageIn<T> sc, const T* __restrict__ Ms_b)
{
    using G = XR2C<T, M>;
    constexpr int kE = G::kE, kT = G::kT, kRows = G::kRows;
    constexpr int kL = G::S::kLds;  // LDS slots per row
    __shared__ cx<T> lds[kRows * kL];
    const int t = threadIdx.x % kT, rl = threadIdx.x / kT;
    const long row = (long)blockIdx.x * kRows + rl;
    const bool valid = row < (long)nrows * ncomp;
    const long c = valid ? row / nrows : 0, r = valid ? row % nrows : 0;
    const long base = c * in_comp + r * in_row;
    const T* src = in + base;
    const T* msrc = PERCELL ? Ms_cell + r * in_row : nullptr;
    if (!PERCELL && Ms_b) Ms = Ms_b[(int)c / 3];
    T cj[7];
    double ej[7];
    if constexpr (COMB) {
        const double hs = sc.h ? *sc.h : 1.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            cj[j] = (T)(sc.c[j] * hs);
            ej[j] = sc.e[j] * hs;
        }
    }
    cx<T> v[kE];
    if (MMX_XVEC && vec) {
        // n_in even and every row start aligned to two reals: one paired load
        // per element (x[2n], x[2n+1])
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int n = t + q * kT;
            cx<T> ab = {0, 0};
            if (!(HALF && q >= kE / 2) && valid && 2 * n < n_in) {
                ab = *reinterpret_cast<const cx<T>*>(src + 2 * n);
                if constexpr (COMB) {
                    const long o = base + 2 * n;
                    double e0 = 0.0, e1 = 0.0;
#pragma unroll
                    for (int j = 0; j < 7; ++j) {
                        const bool uc = sc.c[j] != 0.0, ue = sc.ep && sc.e[j] != 0.0;
                        if (!uc && !ue) continue;
                        const cx<T> kv = *reinterpret_cast<const cx<T>*>(sc.k[j] + o);
                        if (uc) {
                            ab.x += cj[j] * kv.x;
                            ab.y += cj[j] * kv.y;
                        }
                        if (ue) {
                            e0 += ej[j] * (double)kv.x;
                            e1 += ej[j] * (double)kv.y;
                        }
                    }
                    *reinterpret_cast<cx<T>*>(sc.ys + o) = ab;
                    if (sc.ep) *reinterpret_cast<cx<T>*>(sc.ep + o) = cx<T>{(T)e0, (T)e1};
                }
                if (PERCELL) {
                    const cx<T> mm = *reinterpret_cast<const cx<T>*>(msrc + 2 * n);
                    ab = {ab.x * mm.x, ab.y * mm.y};
                } else {
                    ab = {ab.x * Ms, ab.y * Ms};
                }
            }
            v[q] = ab;
        }
    } else {
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int n = t + q * kT;  // first-stage input index
            const int i0 = 2 * n, i1 = 2 * n + 1;
            T a = 0, b = 0;
            // HALF: n_in <= M, so inputs q >= kE/2 (n >= M/2) are zero padding
            if (!(HALF && q >= kE / 2)) {
                if constexpr (COMB) {
                    if (valid && i0 < n_in) a = stage_elem(sc, cj, ej, base + i0) * (PERCELL ? msrc[i0] : Ms);
                    if (valid && i1 < n_in) b = stage_elem(sc, cj, ej, base + i1) * (PERCELL ? msrc[i1] : Ms);
                } else {
                    if (valid && i0 < n_in) a = src[i0] * (PERCELL ? msrc[i0] : Ms);
                    if (valid && i1 < n_in) b = src[i1] * (PERCELL ? msrc[i1] : Ms);
                }
            }
            v[q] = {a, b};
        }
    }
    cx<T>* L = lds + rl * kL;
    WgFFT<T, M, Regs<T>::x, -1, HALF>::run(v, t, L, 1, tw, Lmax / M);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kE; ++q) L[G::S::out_index(t, q)] = v[q];
    __syncthreads();
    if (!valid) return;
    cx<T>* dst = out + c * out_comp + r * out_row;
    const int tws = Lmax / (2 * M);
#pragma unroll
    for (int q = 0; q < kE; ++q) {
        const int k = t + q * kT;
        const cx<T> A = L[k], B = cconj(L[(M - k) & (M - 1)]);
        const cx<T> S = {(T)0.5 * (A.x + B.x), (T)0.5 * (A.y + B.y)};
        const cx<T> D = {(T)0.5 * (A.x - B.x), (T)0.5 * (A.y - B.y)};
        const cx<T> wD = cmul(tw[k * tws], D);
        dst[k] = {S.x + wD.y, S.y - wD.x};  // S - i wD
    }
    if (t == 0) {
        const cx<T> Z0 = L[0];
        dst[M] = {Z0.x - Z0.y, (T)0};
    }
}

// Element idx of a uniformly addressed array.  O32: idx * sizeof(P) is below
// 4 GiB, and the access becomes a scalar base plus a 32-bit vector byte
// offset (no 64-bit address arithmetic per access).
template <bool O32, typename P, typename I>
__device__ __forceinline__ P& elem(P* base, I idx)
{
    if constexpr (O32)
        return *reinterpret_cast<P*>(reinterpret_cast<char*>(base) +
                                     (unsigned)idx * (unsigned)sizeof(P));
    else
        return base[idx];
}
template <bool O32, typename P, typename I>
__device__ __forceinline__ const P& elem(const P* base, I idx)
{
    if constexpr (O32)
        return *reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) +
                                           (unsigned)idx * (unsigned)sizeof(P));
    else
        return base[idx];
}

// ---------------------------------------------------------------------------
// F2 / I2 (and the kernel set-up): batched strided complex transforms.
// A block owns B adjacent columns (contiguous in memory) of one pencil group;
// element e of column col sits at base + e*es + col.  Loads e < n_in (zeros
// beyond), stores e < n_out.
// ---------------------------------------------------------------------------
template <typename T, int L>
struct Strided {
    using S = FFTShape<L, Regs<T>::s>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kB = cmin(64, cmax(1, MMX_SBLOCK / kT));
};

// HALF (forward): n_in <= L/2, the upper half of the inputs is zero padding.
// HALF (inverse): n_out <= L/2, outputs e >= L/2 are never stored.
// O32: every element offset of `in` and `out` times its size is below 4 GiB
// (32-bit index arithmetic, scalar base + vector byte offset accesses).
template <typename T, int L, int DIR, bool HALF, bool O32>
__global__ __launch_bounds__((Strided<T, L>::kB * Strided<T, L>::kT)) MMX_STRIDED_ATTR void k_strided(
    const cx<T>* in, cx<T>* out, int n_in, int n_out, long es_in, long es_out, int ncols,
    int ntile, int G2, long nblocks, long g1_in, long g1_out, long g2_in, long g2_out,
    const cx<T>* __restrict__ tw, int Lmax)
{
    using I = typename std::conditional<O32, unsigned, long>::type;
    using G = Strided<T, L>;
    constexpr int kE = G::kE, kT = G::kT, kB = G::kB;
    constexpr bool HIN = HALF && DIR < 0, HOUT = HALF && DIR > 0;
    constexpr bool SPL = MMX_SSPLIT != 0;
    // complex slots, or (SPL) real slots in half of the same array
    __shared__ cx<T> lds[G::S::kStages > 1 ? (SPL ? (kB * G::S::kLds + 1) / 2 : kB * G::S::kLds) : 1];
    const long lb = xcd_logical();
    if (lb >= nblocks) return;
    const int tile = (int)(lb % ntile);
    const long rest = lb / ntile;
    const long g2 = rest % G2, g1 = rest / G2;
    const int b = threadIdx.x % kB, t = threadIdx.x / kB;
    const int col = tile * kB + b;
    const bool cv = col < ncols;
    const I so = (I)g1 * (I)g1_in + (I)g2 * (I)g2_in + (I)col;
    const I dof = (I)g1 * (I)g1_out + (I)g2 * (I)g2_out + (I)col;
    cx<T> v[kE];
#pragma unroll
    for (int r = 0; r < kE; ++r) {
        const int e = t + r * kT;
        v[r] = (!(HIN && r >= kE / 2) && cv && e < n_in) ? elem<O32>(in, so + (I)e * (I)es_in)
                                                          : cx<T>{0, 0};
    }
    cx<T>* lb_ = SPL ? reinterpret_cast<cx<T>*>(reinterpret_cast<T*>(lds) + b) : lds + b;
    WgFFT<T, L, Regs<T>::s, DIR, HIN, SPL>::run(v, t, lb_, kB, tw, Lmax / L);
    if (!cv) return;
    constexpr int Rl = G::S::kLast;
#pragma unroll
    for (int i = 0; i < kE; ++i) {
        if (HOUT && (i % Rl) >= Rl / 2) continue;  // e >= L/2
        const int e = G::S::out_index(t, i);
        if (e < n_out) elem<O32>(out, dof + (I)e * (I)es_out) = v[i];
    }
}

// ---------------------------------------------------------------------------
// F3 (and the single-layer y pass): forward transform of all three
// components along the last padded axis, product with the folded real
// spectral kernel, inverse transform, store the first n_valid elements.
// AXIS = 2: pencils along z, group g = ky.  AXIS = 1: pencils along y (Pz=1).
// ---------------------------------------------------------------------------
template <typename T, int L>
struct Mid {
    static constexpr int kRegs = Regs<T>::mid;
    using S = FFTShape<L, kRegs>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kB =
        cmin(64, cmax(1, (sizeof(T) == 4 ? MMX_MBLOCK : MMX_MBLOCK_F64) / kT));
};

// One pencil group (fixed ky for AXIS = 2) of the last-axis pass: load three
// components, forward transform, product with the spectral kernel, inverse
// transform, store.  HALF: n_valid <= L/2 (always true with zero padding).
// Element (c, e) of the group is S[o + c*cs + e*es]; index arithmetic is done
// in 32 bits when O32.  PROD 0: the symmetric demag product with the six
// folded real components; PROD 1: the Oersted product h = j x (i g) with the
// three folded components g (imaginary spectrum, odd along its own axis).
// G: the thread shape (kE registers, kT threads per transform); the
// transform's LDS scratch is lds[s * lstride].  WAVE: the kT threads of a
// transform share one wavefront (exchanges without workgroup barriers).
// The folded spectral kernel read from global memory: component c at the
// folded indices (kyf, kzf) of column col.
template <typename T, bool O32>
struct KGlobal {
    using I = typename std::conditional<O32, unsigned, long>::type;
    const T* __restrict__ K;
    I Kn, plane, Hxp, col;
    __device__ __forceinline__ T operator()(int c, int kyf, int kzf) const
    {
        return elem<O32>(K, (I)c * Kn + (I)kzf * plane + (I)kyf * Hxp + col);
    }
};

// KG: the kernel accessor kget(c, kyf, kzf) (c = component, kyf/kzf the
// folded y and z indices; the sign flips are applied here).
// Load the three components of one column of the group: v[c][r] = element
// t + r*kT (zero beyond n_valid, in the upper half with HALF, or for !cv).
template <typename G, typename T, bool HALF, bool O32>
__device__ __forceinline__ void mid_load(cx<T> (&v)[3][G::kE], const cx<T>* S, long o_,
                                         int n_valid, long es_, long cs_, bool cv, int t)
{
    using I = typename std::conditional<O32, unsigned, long>::type;
    constexpr int kE = G::kE, kT = G::kT;
    const I o = (I)o_, es = (I)es_, cs = (I)cs_;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < kE; ++r) {
            const int e = t + r * kT;
            v[c][r] = (!(HALF && r >= kE / 2) && cv && e < n_valid)
                          ? elem<O32>(S, o + (I)c * cs + (I)e * es)
                          : cx<T>{0, 0};
        }
}

// Transform, product and inverse of one column loaded by mid_load, then the
// store of the first n_valid elements.
template <typename G, bool WAVE, typename T, int L, int AXIS, bool HALF, bool O32, int PROD,
          typename KG>
__device__ __forceinline__ void mid_group(cx<T> (&v)[3][G::kE], cx<T>* S, long o_,
                                          const KG& kget, int n_valid, long es_, long cs_,
                                          bool cv, int g, int t, cx<T>* lds, int lstride, int Py,
                                          int Pz, const cx<T>* __restrict__ tw, int twstride)
{
    using I = typename std::conditional<O32, unsigned, long>::type;
    constexpr int kE = G::kE, kT = G::kT;
    constexpr int kRE = G::kRegs;
    const I o = (I)o_, es = (I)es_, cs = (I)cs_;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        WgFFT<T, L, kRE, -1, HALF, false, WAVE>::run(v[c], t, lds, lstride, tw, twstride);

    if (cv) {
        const int hy = Py / 2, hz = Pz / 2;
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            const int kk = G::S::out_index(t, i);
            int ky, kz;
            if constexpr (AXIS == 2) {
                kz = kk;
                ky = g;
            } else {
                ky = kk;
                kz = 0;
            }
            const bool fy = ky > hy, fz = kz > hz;
            const int kyf = fy ? Py - ky : ky, kzf = fz ? Pz - kz : kz;
            const T sy = fy ? (T)-1 : (T)1, sz = fz ? (T)-1 : (T)1;
            if constexpr (PROD == 1) {
                const T gx = kget(0, kyf, kzf), gy = sy * kget(1, kyf, kzf);
                const T gz = sz * kget(2, kyf, kzf);
                const cx<T> jx = v[0][i], jy = v[1][i], jz = v[2][i];
                // c = j x g, h = i c = (-c.im, c.re)
                const cx<T> c0 = {jy.x * gz - jz.x * gy, jy.y * gz - jz.y * gy};
                const cx<T> c1 = {jz.x * gx - jx.x * gz, jz.y * gx - jx.y * gz};
                const cx<T> c2 = {jx.x * gy - jy.x * gx, jx.y * gy - jy.y * gx};
                v[0][i] = {-c0.y, c0.x};
                v[1][i] = {-c1.y, c1.x};
                v[2][i] = {-c2.y, c2.x};
                continue;
            }
            const T kxx = kget(0, kyf, kzf), kyy = kget(1, kyf, kzf);
            const T kzz = kget(2, kyf, kzf);
            const T kxy = sy * kget(3, kyf, kzf), kxz = sz * kget(4, kyf, kzf);
            const T kyz = sy * sz * kget(5, kyf, kzf);
            const cx<T> mx = v[0][i], my = v[1][i], mz = v[2][i];
            v[0][i] = {kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y};
            v[1][i] = {kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y};
            v[2][i] = {kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y};
        }
    }
    // The forward outputs of thread t are exactly the inverse inputs
    // t + m*kT; only their register order differs.
    constexpr int Rl = G::S::kLast;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<T> w[kE];
#pragma unroll
        for (int i = 0; i < kE; ++i) w[i / Rl + (i % Rl) * (kE / Rl)] = v[c][i];
#pragma unroll
        for (int i = 0; i < kE; ++i) v[c][i] = w[i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        WgFFT<T, L, kRE, 1, false, false, WAVE>::run(v[c], t, lds, lstride, tw, twstride);
    if (!cv) return;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            if (HALF && (i % Rl) >= Rl / 2) continue;  // e >= L/2
            const int e = G::S::out_index(t, i);
            if (e < n_valid) elem<O32>(S, o + (I)c * cs + (I)e * es) = v[c][i];
        }
}

// AXIS = 2: pencils along z; a block owns the column tile at ky = g and, for
// 0 < g < Py/2, also ky = Py - g, which uses the same (folded) rows of the
// spectral kernel.  ADJ: the two groups go to adjacent blocks instead (same
// XCD, same time), so the second read of each kernel row is an L2 hit rather
// than a re-read after the rows have left L2.  AXIS = 1: pencils along y
// (single layer), one group.  O32: spectra and kernel arrays below 4 GiB.
template <typename T, int L, int AXIS, bool HALF, bool O32, bool ADJ, int PROD = 0>
__global__ __launch_bounds__((Mid<T, L>::kB * Mid<T, L>::kT)) void k_mid(
    cx<T>* S, const T* __restrict__ Khat, int n_valid, long es, long cs, long gstride, int ncols,
    int ntile, long nblocks, int Py, int Pz, long Kn, int Hxp, const cx<T>* __restrict__ tw,
    int Lmax)
{
    using G = Mid<T, L>;
    constexpr int kB = G::kB;
    __shared__ cx<T> lds[G::S::kStages > 1 ? kB * G::S::kLds : 1];
    const long lb = xcd_logical();
    if (lb >= nblocks) return;
    int tile, g;
    bool paired;
    if constexpr (ADJ) {
        const int which = (int)(lb & 1);
        const long rest = lb >> 1;
        tile = (int)(rest % ntile);
        const int gp = (int)(rest / ntile);
        if (which && (gp == 0 || 2 * gp == Py)) return;  // its own mirror
        g = which ? Py - gp : gp;
        paired = false;
    } else {
        tile = (int)(lb % ntile);
        g = (int)(lb / ntile);
        paired = AXIS == 2 && g > 0 && 2 * g < Py;
    }
    const int b = threadIdx.x % kB, t = threadIdx.x / kB;
    const int col = tile * kB + b;
    const bool cv = col < ncols;
    using I = typename KGlobal<T, O32>::I;
    const KGlobal<T, O32> kg{Khat, (I)Kn, (I)((long)(Py / 2 + 1) * Hxp), (I)Hxp, (I)col};
    {
        cx<T> v[3][G::kE];
        mid_load<G, T, HALF, O32>(v, S, (long)g * gstride + col, n_valid, es, cs, cv, t);
        mid_group<G, false, T, L, AXIS, HALF, O32, PROD>(v, S, (long)g * gstride + col, kg,
                                                         n_valid, es, cs, cv, g, t, lds + b, kB,
                                                         Py, Pz, tw, Lmax / L);
    }
    if (paired) {
        const int g2 = Py - g;
        cx<T> v[3][G::kE];
        mid_load<G, T, HALF, O32>(v, S, (long)g2 * gstride + col, n_valid, es, cs, cv, t);
        mid_group<G, false, T, L, AXIS, HALF, O32, PROD>(v, S, (long)g2 * gstride + col, kg,
                                                         n_valid, es, cs, cv, g2, t, lds + b, kB,
                                                         Py, Pz, tw, Lmax / L);
    }
}

// Wave-local shape of the last-axis pass: kT = L/kE threads per transform,
// all in one wavefront (lane = t * kCB + b), kCB column transforms per
// wavefront, kW wavefronts per block.  Lengths whose transform would need
// more than 64 threads use k_mid.
template <typename T, int L>
struct MidW {
    static constexpr int kRegs = sizeof(T) == 4 ? MMX_RMW_F32 : MMX_RMW_F64;
    using S = FFTShape<L, kRegs>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr bool kOK = kT <= 64;
    static constexpr int kCB = kOK ? 64 / kT : 1;
    static constexpr int kW = 2;  // AXIS = 2: the wavefronts of ky and Py - ky
};

// The block's folded kernel tile staged in LDS: component c at the folded
// index r along the transform axis (kzf for AXIS = 2, kyf for AXIS = 1) of
// column b of the tile, at t[(c * R + r) * CB + b].
template <typename T, int AXIS, int R, int CB>
struct KLds {
    const T* t;
    int b;
    __device__ __forceinline__ T operator()(int c, int kyf, int kzf) const
    {
        return t[(c * R + (AXIS == 2 ? kzf : kyf)) * CB + b];
    }
};

// F3 with wave-local transforms.  The block first stages what its
// wavefronts read besides their own spectra -- the folded kernel rows of its
// column tile(s) and the twiddles of length L -- in LDS, in the same memory
// phase as the spectrum loads, so the transforms and the product run without
// waiting on global memory; after that one barrier the wavefronts run on
// their own (no further workgroup barrier).  AXIS = 2: the block holds the
// column tile tb of the pair ky = gp (wavefront 0) and ky = Py - gp
// (wavefront 1), which share the folded kernel rows.  AXIS = 1 (single
// layer, one group): each wavefront its own column tile.  A batch of nbatch
// requests (spectra bstride complex values apart, one kernel) takes nbatch
// times the blocks, request-major.
template <typename T, int L, int AXIS, bool HALF, bool O32, int PROD>
__global__ __launch_bounds__((64 * MidW<T, L>::kW)) MMX_MIDW_ATTR void k_mid_w(
    cx<T>* S, const T* __restrict__ Khat, int n_valid, long es, long cs, long gstride, int ncols,
    int ntb, long nblocks, int Py, int Pz, long Kn, int Hxp, const cx<T>* __restrict__ tw,
    int Lmax, int nbatch, long bstride)
{
    using G = MidW<T, L>;
    constexpr int kCB = G::kCB, kW = G::kW;
    constexpr int NK = PROD == 0 ? 6 : 3;        // kernel components
    constexpr int R = L / 2 + 1;                  // folded rows along the transform axis
    constexpr int NT = AXIS == 2 ? 1 : kW;        // column tiles per block
    constexpr int KT = NK * R * kCB;              // kernel values per tile
    __shared__ T kt[NT * KT];
    __shared__ cx<T> twl[L];
    __shared__ cx<T> lds[kW][G::S::kStages > 1 ? kCB * G::S::kLds : 1];
    long lb = xcd_logical();
    if (nbatch > 1) {
        if (lb >= nblocks * nbatch) return;
        const long bi = lb / nblocks;
        lb -= bi * nblocks;
        S += bi * bstride;
    } else if (lb >= nblocks) {
        return;  // uniform over the block
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tile0, g, gp = 0;
    bool active = true;
    if constexpr (AXIS == 2) {
        const int tb = (int)(lb % ntb);
        gp = (int)(lb / ntb);
        tile0 = tb;
        const bool mirror = wave & 1;
        if (mirror && (gp == 0 || 2 * gp >= Py)) active = false;  // its own mirror
        g = mirror ? Py - gp : gp;
    } else {
        tile0 = (int)lb * kW;
        g = 0;
    }
    const int tile = AXIS == 2 ? tile0 : tile0 + wave;
    const int b = lane % kCB, t = lane / kCB;
    const int col = tile * kCB + b;
    const bool cv = active && col < ncols;
    // one memory phase: the kernel tile(s) and twiddles for LDS, then the
    // spectrum column (every thread of the block takes part in the staging).
    // Staging: thread (rr, bb) = (tid / kCB, tid % kCB) takes rows rr, rr + RCH,
    // ... of every component; offsets other than its own are uniform.
    using I = typename std::conditional<O32, unsigned, long>::type;
    const I plane = (I)(Py / 2 + 1) * (I)Hxp;
    constexpr int RCH = 64 * kW / kCB;              // rows per staging round
    constexpr int NCH = (R + RCH - 1) / RCH;         // rounds per component
    constexpr int NQ = NT * NK * NCH;
    constexpr int NTW = (L + 64 * kW - 1) / (64 * kW);
    const int rr = (int)threadIdx.x / kCB, bb = (int)threadIdx.x % kCB;
    T kv[NQ];
#pragma unroll
    for (int tl = 0; tl < NT; ++tl) {
        const int cl = (tile0 + tl) * kCB + bb;
        const I base = (AXIS == 2 ? (I)rr * plane + (I)gp * (I)Hxp : (I)rr * (I)Hxp) + (I)cl;
        const I rstep = AXIS == 2 ? (I)RCH * plane : (I)RCH * (I)Hxp;
#pragma unroll
        for (int c = 0; c < NK; ++c)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const bool use = cl < ncols && ch * RCH + rr < R;
                kv[(tl * NK + c) * NCH + ch] =
                    use ? elem<O32>(Khat, base + (I)c * (I)Kn + (I)ch * rstep) : (T)0;
            }
    }
    const int tws = Lmax / L;
    cx<T> twv[NTW];
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = q * 64 * kW + (int)threadIdx.x;
        twv[q] = n < L ? tw[n * tws] : cx<T>{0, 0};
    }
    cx<T> v[3][G::kE];
    mid_load<G, T, HALF, O32>(v, S, (long)g * gstride + col, n_valid, es, cs, cv, t);
#pragma unroll
    for (int tl = 0; tl < NT; ++tl)
#pragma unroll
        for (int c = 0; c < NK; ++c)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch * RCH + rr < R)
                    kt[tl * KT + (c * R + ch * RCH) * kCB + (int)threadIdx.x] =
                        kv[(tl * NK + c) * NCH + ch];
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = q * 64 * kW + (int)threadIdx.x;
        if (n < L) twl[n] = twv[q];
    }
    __syncthreads();
    if (!active || tile * kCB >= ncols) return;  // from here on, no workgroup barrier
    const KLds<T, AXIS, R, kCB> kg{kt + (AXIS == 2 ? 0 : wave * KT), b};
    mid_group<G, true, T, L, AXIS, HALF, O32, PROD>(v, S, (long)g * gstride + col, kg, n_valid,
                                                    es, cs, cv, g, t, lds[wave] + b, kCB, Py, Pz,
                                                    twl, 1);
}

// ---------------------------------------------------------------------------
// I1: x complex-to-real transform + local field terms + LLG right-hand side.
// ---------------------------------------------------------------------------
struct LocalParams {
    int nx, ny, nz;
    long N;
    long s1_comp;     // nz*ny*Hxp
    int Hxp;
    int with_demag, with_exch, with_anis, with_zee;
    double Ms;        // uniform Ms (ignored with per-cell Ms)
    double exch;      // 2 A / mu0 (divided by Ms_i per cell)
    double idx2, idy2, idz2;  // 1/dx^2 ...
    double anis;      // 2 Ku / mu0 (divided by Ms_i per cell)
    double eu[3];
    int with_anis_hi;  // higher-order anisotropy present
    double anis2;     // 4 Ku2 / mu0
    double cub1, cub2;  // 2 Kc1 / mu0, 2 Kc2 / mu0
    double ec[3][3];  // cubic principal axes
    int with_oe;      // Oersted term present (h_oe)
    double oe_scale;  // its time factor
    int with_dmi;     // DMI term present
    double dmi;       // 2 D / mu0, or 2 / mu0 with per-cell D (divided by Ms_i per cell)
    double edmi[3][3];  // DMI vector of axis k divided by 2 Delta_k
    double H[3];      // uniform external field
    double Hd[3];     // drive field at time t on masked cells
    double gp;        // gamma / (1 + alpha^2)
    double alpha;
    int precess;
};

template <typename T, int M>
struct XC2R {
    static constexpr int Mf = M > 0 ? M : 1;
    using S = FFTShape<Mf, Regs<T>::x1>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kL = S::kLds;  // LDS slots per (row, component) >= Mf
    static constexpr int kRows =
        cmax(1, (sizeof(T) == 4 ? MMX_X1BLOCK : MMX_X1BLOCK_F64) / (3 * kT));
};

__device__ inline void atomic_max_nonneg(double* addr, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// Inverse real x transform of kRows rows (j0 .. j0+kRows-1 at slab k) of
// three components from the spectrum S1 into LDS: component c of row rl ends
// as reals at lds + (rl*3 + c)*kL (x = 0 .. 2M-1, only x < M written).
// 2M-point real inverse via an M-point complex inverse of
//   2 Z[n] = (X[n] + conj X[M-n]) + i w^-n (X[n] - conj X[M-n]).
// Contains barriers: every thread of the block must call it.
template <typename T, int M>
__device__ __forceinline__ void x_c2r_rows(const cx<T>* __restrict__ S1, cx<T>* lds, int k, int j0,
                                           int ny, long s1_comp, int Hxp,
                                           const cx<T>* __restrict__ tw, int Lmax)
{
    using G = XC2R<T, M>;
    if constexpr (M >= 2) {
        constexpr int kE = G::kE, kT = G::kT, kRows = G::kRows, kL = G::kL;
        const int t = threadIdx.x % kT;
        const int c = (threadIdx.x / kT) % 3;
        const int rl = threadIdx.x / (3 * kT);
        const int j = j0 + rl;
        const bool valid = rl < kRows && j < ny;
        const cx<T>* X = S1 + c * s1_comp + ((long)k * ny + (valid ? j : 0)) * Hxp;
        const int tws = Lmax / (2 * M);
        cx<T> v[kE];
#pragma unroll
        for (int r = 0; r < kE; ++r) {
            const int n = t + r * kT;
            cx<T> z = {0, 0};
            if (valid) {
                const cx<T> a = X[n], bb = X[M - n];
                const cx<T> D = {a.x - bb.x, a.y + bb.y};
                const cx<T> wD = cmulc(D, tw[n * tws]);
                z = {a.x + bb.x - wD.y, a.y - bb.y + wD.x};
            }
            v[r] = z;
        }
        cx<T>* L = lds + (rl * 3 + c) * kL;
        WgFFT<T, M, Regs<T>::x1, 1>::run(v, t, L, 1, tw, Lmax / M);
        __syncthreads();
        T* hd = reinterpret_cast<T*>(L);
        constexpr int Rl = G::S::kLast;
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            // outputs n >= M/2 are cells x >= M >= nx: never used
            if ((i % Rl) >= Rl / 2) continue;
            const int e = G::S::out_index(t, i);
            hd[2 * e] = v[i].x;
            hd[2 * e + 1] = v[i].y;
        }
        __syncthreads();
    }
}

// Demag value of component c at cell i of row rl after x_c2r_rows (or, for a
// single cell along x, straight from the spectrum).
template <typename T, int M>
__device__ __forceinline__ T x_c2r_value(const cx<T>* __restrict__ S1, const cx<T>* lds, int rl,
                                         int c, int i, int k, int j, int ny, long s1_comp, int Hxp)
{
    using G = XC2R<T, M>;
    if constexpr (M >= 2) {
        const T* hd = reinterpret_cast<const T*>(lds + (rl * 3 + c) * G::kL);
        return hd[i];
    } else {
        return S1[c * s1_comp + ((long)k * ny + j) * Hxp].x;
    }
}

// 2 a b / (a + b) for a + b != 0, else 0 -- the harmonic-mean coupling of
// the exchange (Sec. 4.2) and of equal-sign DMI strengths (Eq. D_avg).  The
// quotient uses the hardware reciprocal (FP32: 1 ulp; FP64: refined) instead
// of the correctly rounded division sequence.
template <typename T>
__device__ __forceinline__ T harmonic2(T a, T b)
{
    const T s = a + b;
    if (s == (T)0) return (T)0;
    if constexpr (!MMX_EXT_RCP) {
        return (T)2 * a * b / s;
    } else if constexpr (sizeof(T) == 4) {
        return (T)2 * a * b * __builtin_amdgcn_rcpf(s);
    } else {
        // hardware reciprocal refined by two Newton steps (error ~1 ulp)
        double r = __builtin_amdgcn_rcp(s);
        r = fma(r, fma(-s, r, 1.0), r);
        r = fma(r, fma(-s, r, 1.0), r);
        return (T)2 * a * b * r;
    }
}

// Effective DMI coupling of two cells (Eq. D_avg): the harmonic mean for
// equal signs, otherwise minus the geometric mean of sqrt(-Da Db) and
// |Da + Db| / 2.
template <typename T>
__device__ __forceinline__ T dmi_avg(T a, T b)
{
    const T ab = a * b;
    if (ab >= (T)0) return harmonic2(a, b);
    return -sqrt(sqrt(-ab) * fabs(a + b) * (T)0.5);
}

// Stencil variant bits: EXT_DMI adds the DMI term (Sec. 4.3); EXT_PA takes
// per-cell exchange constants A_cell with the harmonic-mean coupling (Sec.
// 4.2), P.exch then being 2 / mu0; EXT_PD takes per-cell DMI strengths D_cell
// with the coupling of Eq. D_avg, P.dmi then being 2 / mu0; EXT_MIX adds the
// opposite-sign case of that average (D_cell holds both signs).  Every
// variant but the plain one (EXT 0) reads a per-cell uniaxial constant
// Ku_cell when given one (P.anis then 2 / mu0); EXT_PK alone is the variant
// for a per-cell Ku without the other extensions.
constexpr int EXT_DMI = 1, EXT_PA = 2, EXT_PD = 4, EXT_MIX = 8, EXT_PK = 16;
// EXT_LO (wave-local local pass, FP32, plain stencil): the state is given as
// m + m_lo (two floats, the rounding residual of a double state), and the
// exchange differences are taken as (m_j - m_i) + (m_lo_j - m_lo_i)
constexpr int EXT_LO = 32;

template <typename T, int M, bool PERCELL, int EXT>
__global__ __launch_bounds__((XC2R<T, M>::kRows * 3 * XC2R<T, M>::kT)) void k_x_c2r_local(
    const cx<T>* __restrict__ S1, const T* __restrict__ m, T* __restrict__ h_out,
    T* __restrict__ dm_out, const T* __restrict__ Ms_cell, const unsigned char* __restrict__ mask,
    LocalParams P, double* torque, int njt, long nblocks, const cx<T>* __restrict__ tw, int Lmax,
    const T* __restrict__ A_cell, const T* __restrict__ D_cell, const T* __restrict__ zw,
    const T* __restrict__ h_oe, const T* __restrict__ Ku_cell)
{
    constexpr bool kDMI = EXT & EXT_DMI, kPA = EXT & EXT_PA, kPD = EXT & EXT_PD;
    constexpr bool kMIX = EXT & EXT_MIX;
    using G = XC2R<T, M>;
    constexpr int kRows = G::kRows, kL = G::kL;
    __shared__ cx<T> lds[kRows * 3 * kL];
    const long lb = xcd_logical();
    if (lb >= nblocks) return;
    // z fastest: the blocks of rows (j, k-1), (j, k), (j, k+1) run together
    // on one XCD, so the z neighbours of m come from its L2
    const int k = MMX_X1_KFAST ? (int)(lb % P.nz) : (int)(lb / njt);
    const int j0 = (MMX_X1_KFAST ? (int)(lb / P.nz) : (int)(lb % njt)) * kRows;
    const int nx = P.nx, ny = P.ny;

    if (P.with_demag) x_c2r_rows<T, M>(S1, lds, k, j0, ny, P.s1_comp, P.Hxp, tw, Lmax);

    const long N = P.N;
    const T exch = (T)P.exch, anis = (T)P.anis;
    const T ix2 = (T)P.idx2, iy2 = (T)P.idy2, iz2 = (T)P.idz2;
    // z couplings of this block's layer: exchange to the layer below / above
    // and the DMI difference scale (equal layers: 1/dz^2, 1/dz^2 and 1, the
    // DMI vector of z being divided by 2 dz already; thin layers of unequal
    // height: 2/(dz_k (dz_k + dz_k-+1)) and 1/(2 dz_k))
    T wz_dn = iz2, wz_up = iz2, dz_s = (T)1;
    if (zw) {
        wz_dn = zw[4 * k];
        wz_up = zw[4 * k + 1];
        dz_s = zw[4 * k + 2];
    }
    const T eux = (T)P.eu[0], euy = (T)P.eu[1], euz = (T)P.eu[2];
    double tmax = 0.0;
    for (int idx = threadIdx.x; idx < kRows * nx; idx += blockDim.x) {
        const int rl = idx / nx, i = idx - rl * nx;
        const int j = j0 + rl;
        if (j >= ny) continue;
        const long cell = i + (long)nx * (j + (long)ny * k);
        const T ms = PERCELL ? Ms_cell[cell] : (T)P.Ms;
        T hx = 0, hy = 0, hz = 0;
        const T mx = m[cell], my = m[N + cell], mz = m[2 * N + cell];
        if (ms != (T)0) {
            if (P.with_demag) {
                hx = x_c2r_value<T, M>(S1, lds, rl, 0, i, k, j, ny, P.s1_comp, P.Hxp);
                hy = x_c2r_value<T, M>(S1, lds, rl, 1, i, k, j, ny, P.s1_comp, P.Hxp);
                hz = x_c2r_value<T, M>(S1, lds, rl, 2, i, k, j, ny, P.s1_comp, P.Hxp);
            }
            const T inv_ms = (T)1 / ms;
            if (EXT != 0 || P.with_exch) {
                // One pass over the six neighbours serves exchange and DMI,
                // free of branches around loads: an absent neighbour reads
                // the cell itself with weight 0.
                T ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
                T Ai = 0, Di = 0;
                if constexpr (kPA) Ai = A_cell[cell];
                if constexpr (kPD) Di = D_cell[cell];
#pragma unroll
                for (int nbi = 0; nbi < 6; ++nbi) {
                    const int dir = nbi >> 1;
                    const bool plus = nbi & 1;
                    const bool has = dir == 0 ? (plus ? i + 1 < nx : i > 0)
                                   : dir == 1 ? (plus ? j + 1 < ny : j > 0)
                                              : (plus ? k + 1 < P.nz : k > 0);
                    const long off = dir == 0 ? 1L : dir == 1 ? (long)nx : (long)nx * ny;
                    const long q = has ? (plus ? cell + off : cell - off) : cell;
                    const T qx = m[q], qy = m[N + q], qz = m[2 * N + q];
                    const bool ok = has && (!PERCELL || Ms_cell[q] != (T)0);
                    T wq = ok ? (dir == 0 ? ix2 : dir == 1 ? iy2 : plus ? wz_up : wz_dn) : (T)0;
                    if constexpr (kPA) wq *= harmonic2(Ai, A_cell[q]);
                    ax += wq * (qx - mx);
                    ay += wq * (qy - my);
                    az += wq * (qz - mz);
                    if constexpr (kDMI) {
                        // D~ (e^dmi_k x m_{i+k}) / (2 Delta_k), e^dmi_{-k} = -e^dmi_k
                        T c = ok ? (plus ? (T)1 : (T)-1) : (T)0;
                        if (dir == 2) c *= dz_s;
                        if constexpr (kMIX)
                            c *= dmi_avg(Di, D_cell[q]);
                        else if constexpr (kPD)
                            c *= harmonic2(Di, D_cell[q]);
                        const T ex = c * (T)P.edmi[dir][0], ey = c * (T)P.edmi[dir][1],
                                ez = c * (T)P.edmi[dir][2];
                        bx += ey * qz - ez * qy;
                        by += ez * qx - ex * qz;
                        bz += ex * qy - ey * qx;
                    }
                }
                const T ce = P.with_exch ? exch * inv_ms : (T)0;
                hx += ce * ax;
                hy += ce * ay;
                hz += ce * az;
                if constexpr (kDMI) {
                    const T cd = (T)P.dmi * inv_ms;
                    hx += cd * bx;
                    hy += cd * by;
                    hz += cd * bz;
                }
            }
            if (P.with_anis) {
                const T em = eux * mx + euy * my + euz * mz;
                // per-cell Ku (extended variants only): P.anis is then 2 / mu0
                T ka = anis;
                if constexpr (EXT != 0)
                    if (Ku_cell) ka *= Ku_cell[cell];
                const T ca = ka * inv_ms * em;
                hx += ca * eux;
                hy += ca * euy;
                hz += ca * euz;
                if (P.with_anis_hi) {
                    // second-order uniaxial: 4 Ku2 (e.m)^3 e / (mu0 Ms)
                    const T cb = (T)P.anis2 * inv_ms * em * em * em;
                    hx += cb * eux;
                    hy += cb * euy;
                    hz += cb * euz;
                    // cubic, in the principal axes c_i: -2 Kc1 m_i (m_j^2 + m_k^2)
                    // - 2 Kc2 m_i m_j^2 m_k^2, over mu0 Ms, mapped back along c_i
                    T pr[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        pr[a] = (T)P.ec[a][0] * mx + (T)P.ec[a][1] * my + (T)P.ec[a][2] * mz;
                    const T q0 = pr[0] * pr[0], q1 = pr[1] * pr[1], q2 = pr[2] * pr[2];
                    const T c1 = (T)P.cub1 * inv_ms, c2 = (T)P.cub2 * inv_ms;
                    const T g0 = -(c1 * pr[0] * (q1 + q2) + c2 * pr[0] * q1 * q2);
                    const T g1 = -(c1 * pr[1] * (q2 + q0) + c2 * pr[1] * q2 * q0);
                    const T g2 = -(c1 * pr[2] * (q0 + q1) + c2 * pr[2] * q0 * q1);
                    hx += g0 * (T)P.ec[0][0] + g1 * (T)P.ec[1][0] + g2 * (T)P.ec[2][0];
                    hy += g0 * (T)P.ec[0][1] + g1 * (T)P.ec[1][1] + g2 * (T)P.ec[2][1];
                    hz += g0 * (T)P.ec[0][2] + g1 * (T)P.ec[1][2] + g2 * (T)P.ec[2][2];
                }
            }
            if (P.with_oe) {
                const T so = (T)P.oe_scale;
                hx += so * h_oe[cell];
                hy += so * h_oe[N + cell];
                hz += so * h_oe[2 * N + cell];
            }
            if (P.with_zee) {
                hx += (T)P.H[0];
                hy += (T)P.H[1];
                hz += (T)P.H[2];
                if (mask && mask[cell]) {
                    hx += (T)P.Hd[0];
                    hy += (T)P.Hd[1];
                    hz += (T)P.Hd[2];
                }
            }
        }
        if (h_out) {
            h_out[cell] = hx;
            h_out[N + cell] = hy;
            h_out[2 * N + cell] = hz;
        }
        // m x h and m x (m x h)
        const T px = my * hz - mz * hy, py = mz * hx - mx * hz, pz = mx * hy - my * hx;
        if (dm_out) {
            const T qx = my * pz - mz * py, qy = mz * px - mx * pz, qz = mx * py - my * px;
            const T gp = (T)P.gp, al = (T)P.alpha, pf = P.precess ? (T)1 : (T)0;
            const bool mag = ms != (T)0;
            dm_out[cell] = mag ? -gp * (pf * px + al * qx) : (T)0;
            dm_out[N + cell] = mag ? -gp * (pf * py + al * qy) : (T)0;
            dm_out[2 * N + cell] = mag ? -gp * (pf * pz + al * qz) : (T)0;
        }
        if (torque && ms != (T)0) {
            const double tq = sqrt((double)px * px + (double)py * py + (double)pz * pz) / (double)ms;
            tmax = tmax > tq ? tmax : tq;
        }
    }
    if (torque) {
        // wavefront max, then one atomic per wavefront
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_down(tmax, off, 64);
            tmax = tmax > o ? tmax : o;
        }
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(torque, tmax);
    }
}

// I1, wave-local form (M >= 2).  A block of 256 threads owns kRB rows
// (j0 .. j0 + kRB - 1) of slab k, laid out M cells apart: thread slot q holds
// cell i = li mod M of row li / M, li = threadIdx.x + 256 q (slots with
// i >= nx idle).  One memory phase first: the spectrum rows for the inverse
// transforms (threads below 3 kRB kT, one transform per kT threads, all in
// one wavefront) and, for every cell, m and its six neighbours (plus the
// per-cell constants of the variant), all with 32-bit offsets from
// per-component bases; then the transforms, whose real outputs go to LDS,
// one barrier, and the local terms from registers.
template <typename T, int M>
struct XC2RW {
    static constexpr int kRegs = Regs<T>::x1;
    using S = FFTShape<(M > 0 ? M : 1), kRegs>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr bool kOK = M >= 2 && kT <= 64;     // a transform fits one wavefront
    static constexpr int kRB = kOK ? cmin(64 / kT, 512 / M) : 1;  // rows per block (kOK)
    static constexpr int kNT = 256;                               // threads per block
    static constexpr int kCPT = kOK ? (kRB * M + kNT - 1) / kNT : 1;
    static constexpr int kLogM = ilog2(M > 0 ? M : 1);
    static_assert(!kOK || 3 * kRB * kT <= kNT, "transform threads exceed the block");
};

// The error-norm accumulation of the last Dormand-Prince stage (ERR): the
// partial error ep from the x forward pass, the state y, the coefficient e6
// of the derivative computed here, the tolerances, and the block partials
// (sums in part[0, nblocks), non-finite counts in part[nblocks, 2 nblocks)).
template <typename T>
struct LocalErr {
    const T* ep;
    const T* y;
    double e6, rtol, atol;
    double* part;
};

// BATCH: nbatch requests of one grid, request-major blocks; request b's
// spectrum, state and outputs follow those of b - 1 (3 components each), its
// material and field constants are Pb[b] and its torque maximum goes to
// torque[b * tstride].  Every address comes from the launch's own geometry
// (Pk: nx, ny, nz, N, s1_comp, Hxp), never from a request's entry.
template <typename T, int M, bool PERCELL, int EXT, bool BATCH, bool ERR = false>
__global__ __launch_bounds__(256) void k_x_c2r_local_w(
    const cx<T>* __restrict__ S1, const T* __restrict__ m, T* __restrict__ h_out,
    T* __restrict__ dm_out, const T* __restrict__ Ms_cell, const unsigned char* __restrict__ mask,
    LocalParams Pk, double* torque, long nblocks, const cx<T>* __restrict__ tw, int Lmax,
    const T* __restrict__ A_cell, const T* __restrict__ D_cell, const T* __restrict__ zw,
    const T* __restrict__ h_oe, const T* __restrict__ Ku_cell,
    const LocalParams* __restrict__ Pb, int nbatch, long tstride, LocalErr<T> E,
    const T* __restrict__ m_lo)
{
    constexpr bool kDMI = EXT & EXT_DMI, kPA = EXT & EXT_PA, kPD = EXT & EXT_PD;
    constexpr bool kMIX = EXT & EXT_MIX, kLO = EXT & EXT_LO;
    using G = XC2RW<T, M>;
    constexpr int kE = G::kE, kT = G::kT, RB = G::kRB, CPT = G::kCPT, kL = G::S::kLds;
    constexpr int NTW = (M + G::kNT - 1) / G::kNT;
    __shared__ cx<T> lds[3 * RB * kL];
    __shared__ cx<T> twl[M];  // the M-point transform's twiddles
    long lb = xcd_logical();
    int bi = 0;
    if constexpr (BATCH) {
        if (lb >= nblocks * nbatch) return;
        bi = (int)(lb / nblocks);
        lb -= (long)bi * nblocks;
        const long n3 = 3 * Pk.N;
        S1 += (long)bi * 3 * Pk.s1_comp;
        m += (long)bi * n3;
        if constexpr (kLO) m_lo += (long)bi * n3;
        if (h_out) h_out += (long)bi * n3;
        if (dm_out) dm_out += (long)bi * n3;
        if (torque) torque += (long)bi * tstride;
    } else {
        if (lb >= nblocks) return;
    }
    const LocalParams& P = BATCH ? Pb[bi] : Pk;
    // z fastest: the blocks of rows (j, k-1), (j, k), (j, k+1) run together
    // on one XCD, so the z neighbours of m come from its L2
    const int nx = Pk.nx, ny = Pk.ny, nz = Pk.nz;
    const int k = (int)((unsigned)lb % (unsigned)nz);
    const int j0 = (int)((unsigned)lb / (unsigned)nz) * RB;
    const int tid = threadIdx.x;
    const unsigned N = (unsigned)Pk.N;
    const unsigned sxy = (unsigned)nx * (unsigned)ny;

    // ---- memory phase: spectrum rows ----
    const bool with_demag = P.with_demag != 0;
    const bool fthr = tid < 3 * RB * kT;
    const int tau = tid / kT, t = tid % kT;
    const int frl = tau / 3, fc = tau % 3;
    const bool frow = with_demag && fthr && j0 + frl < ny;
    cx<T> xa[kE], xb[kE];
    {
        const cx<T>* X =
            S1 + (long)fc * Pk.s1_comp + ((long)k * ny + (frow ? j0 + frl : 0)) * Pk.Hxp;
#pragma unroll
        for (int r = 0; r < kE; ++r) {
            const int n = t + r * kT;
            xa[r] = frow ? X[n] : cx<T>{0, 0};
            xb[r] = frow ? X[M - n] : cx<T>{0, 0};
        }
    }
    cx<T> twv[NTW];
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = tid + G::kNT * q;
        twv[q] = n < M ? tw[n * (Lmax / M)] : cx<T>{0, 0};
    }
    // ---- memory phase: cells and neighbours ----
    const T* mc0 = m;
    const T* mc1 = m + N;
    const T* mc2 = m + 2 * (size_t)N;
    unsigned cell[CPT];
    bool cv[CPT], has[CPT][6];
    unsigned q6[CPT][6];
    T mv[CPT][7][3];
    T mlo[kLO ? CPT : 1][kLO ? 7 : 1][3];
    T msv[CPT][7];
    T Av[CPT][7], Dv[CPT][7];
    int jj[CPT], ii[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int li = tid + G::kNT * q;
        const int rl = li >> G::kLogM, i = li & (M - 1);
        const int j = j0 + rl;
        jj[q] = j;
        ii[q] = i;
        cv[q] = li < RB * M && i < nx && j < ny;
        const unsigned c0 = cv[q] ? (unsigned)i + (unsigned)nx * (unsigned)j + sxy * (unsigned)k : 0u;
        cell[q] = c0;
        // an idle slot (cell 0 stands in) has no neighbours: its offsets
        // must not step off the cell range
        has[q][0] = cv[q] && i > 0;
        has[q][1] = cv[q] && i + 1 < nx;
        has[q][2] = cv[q] && j > 0;
        has[q][3] = cv[q] && j + 1 < ny;
        has[q][4] = cv[q] && k > 0;
        has[q][5] = cv[q] && k + 1 < nz;
        q6[q][0] = has[q][0] ? c0 - 1u : c0;
        q6[q][1] = has[q][1] ? c0 + 1u : c0;
        q6[q][2] = has[q][2] ? c0 - (unsigned)nx : c0;
        q6[q][3] = has[q][3] ? c0 + (unsigned)nx : c0;
        q6[q][4] = has[q][4] ? c0 - sxy : c0;
        q6[q][5] = has[q][5] ? c0 + sxy : c0;
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            const unsigned qq = d == 0 ? c0 : q6[q][d - 1];
            mv[q][d][0] = elem<true>(mc0, qq);
            mv[q][d][1] = elem<true>(mc1, qq);
            mv[q][d][2] = elem<true>(mc2, qq);
            msv[q][d] = PERCELL ? elem<true>(Ms_cell, qq) : (T)P.Ms;
            Av[q][d] = kPA ? elem<true>(A_cell, qq) : (T)0;
            Dv[q][d] = kPD ? elem<true>(D_cell, qq) : (T)0;
            if constexpr (kLO) {
                mlo[q][d][0] = elem<true>(m_lo, qq);
                mlo[q][d][1] = elem<true>(m_lo + N, qq);
                mlo[q][d][2] = elem<true>(m_lo + 2 * (size_t)N, qq);
            }
        }
    }

    // ---- inverse x transforms (three per row, each in one wavefront) ----
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = tid + G::kNT * q;
        if (n < M) twl[n] = twv[q];
    }
    __syncthreads();
    T* hd = reinterpret_cast<T*>(lds + (frl * 3 + fc) * kL);
    if (with_demag && fthr) {
        const int tws = Lmax / (2 * M);
        cx<T> v[kE];
#pragma unroll
        for (int r = 0; r < kE; ++r) {
            const int n = t + r * kT;
            const cx<T> a = xa[r], bb = xb[r];
            const cx<T> D = {a.x - bb.x, a.y + bb.y};
            const cx<T> wD = cmulc(D, tw[n * tws]);
            v[r] = {a.x + bb.x - wD.y, a.y - bb.y + wD.x};
        }
        WgFFT<T, M, G::kRegs, 1, false, false, true>::run(v, t, lds + (frl * 3 + fc) * kL, 1, twl,
                                                          1);
        fft_sync<true>();  // the transform's last exchange reads precede these writes
        constexpr int Rl = G::S::kLast;
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            // outputs n >= M/2 are cells x >= M >= nx: never used
            if ((i % Rl) >= Rl / 2) continue;
            const int e = G::S::out_index(t, i);
            reinterpret_cast<cx<T>*>(hd)[e] = v[i];  // reals 2e, 2e + 1
        }
    }
    __syncthreads();

    // ---- local terms ----
    const T exch = (T)P.exch, anis = (T)P.anis;
    const T ix2 = (T)P.idx2, iy2 = (T)P.idy2, iz2 = (T)P.idz2;
    T wz_dn = iz2, wz_up = iz2, dz_s = (T)1;
    if (zw) {
        wz_dn = zw[4 * k];
        wz_up = zw[4 * k + 1];
        dz_s = zw[4 * k + 2];
    }
    const T eux = (T)P.eu[0], euy = (T)P.eu[1], euz = (T)P.eu[2];
    double tmax = 0.0;
    double eacc = 0.0, ebad = 0.0;  // ERR
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        if (!cv[q]) continue;
        const unsigned c0 = cell[q];
        const int rl = jj[q] - j0, i = ii[q];
        const T ms = msv[q][0];
        const T mx = mv[q][0][0], my = mv[q][0][1], mz = mv[q][0][2];
        T hx = 0, hy = 0, hz = 0;
        if (ms != (T)0) {
            if (with_demag) {
                hx = reinterpret_cast<const T*>(lds + (rl * 3 + 0) * kL)[i];
                hy = reinterpret_cast<const T*>(lds + (rl * 3 + 1) * kL)[i];
                hz = reinterpret_cast<const T*>(lds + (rl * 3 + 2) * kL)[i];
            }
            const T inv_ms = (T)1 / ms;
            if (EXT != 0 || P.with_exch) {
                // one pass over the six neighbours serves exchange and DMI;
                // an absent neighbour holds the cell itself with weight 0
                T ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
                const T Ai = Av[q][0], Di = Dv[q][0];
#pragma unroll
                for (int nbi = 0; nbi < 6; ++nbi) {
                    const int dir = nbi >> 1;
                    const bool plus = nbi & 1;
                    const T qx = mv[q][nbi + 1][0], qy = mv[q][nbi + 1][1], qz = mv[q][nbi + 1][2];
                    const bool ok = has[q][nbi] && (!PERCELL || msv[q][nbi + 1] != (T)0);
                    T wq = ok ? (dir == 0 ? ix2 : dir == 1 ? iy2 : plus ? wz_up : wz_dn) : (T)0;
                    if constexpr (kPA) wq *= harmonic2(Ai, Av[q][nbi + 1]);
                    if constexpr (kLO) {
                        // differences of the split state: the float parts
                        // subtract exactly for neighbouring directions, the
                        // residuals carry the rest of the double state
                        ax += wq * ((qx - mx) + (mlo[q][nbi + 1][0] - mlo[q][0][0]));
                        ay += wq * ((qy - my) + (mlo[q][nbi + 1][1] - mlo[q][0][1]));
                        az += wq * ((qz - mz) + (mlo[q][nbi + 1][2] - mlo[q][0][2]));
                    } else {
                        ax += wq * (qx - mx);
                        ay += wq * (qy - my);
                        az += wq * (qz - mz);
                    }
                    if constexpr (kDMI) {
                        // D~ (e^dmi_k x m_{i+k}) / (2 Delta_k), e^dmi_{-k} = -e^dmi_k
                        T c = ok ? (plus ? (T)1 : (T)-1) : (T)0;
                        if (dir == 2) c *= dz_s;
                        if constexpr (kMIX)
                            c *= dmi_avg(Di, Dv[q][nbi + 1]);
                        else if constexpr (kPD)
                            c *= harmonic2(Di, Dv[q][nbi + 1]);
                        const T ex = c * (T)P.edmi[dir][0], ey = c * (T)P.edmi[dir][1],
                                ez = c * (T)P.edmi[dir][2];
                        bx += ey * qz - ez * qy;
                        by += ez * qx - ex * qz;
                        bz += ex * qy - ey * qx;
                    }
                }
                const T ce = P.with_exch ? exch * inv_ms : (T)0;
                hx += ce * ax;
                hy += ce * ay;
                hz += ce * az;
                if constexpr (kDMI) {
                    const T cd = (T)P.dmi * inv_ms;
                    hx += cd * bx;
                    hy += cd * by;
                    hz += cd * bz;
                }
            }
            if (P.with_anis) {
                const T em = eux * mx + euy * my + euz * mz;
                // per-cell Ku (extended variants only): P.anis is then 2 / mu0
                T ka = anis;
                if constexpr (EXT != 0)
                    if (Ku_cell) ka *= elem<true>(Ku_cell, c0);
                const T ca = ka * inv_ms * em;
                hx += ca * eux;
                hy += ca * euy;
                hz += ca * euz;
                if (P.with_anis_hi) {
                    // second-order uniaxial: 4 Ku2 (e.m)^3 e / (mu0 Ms)
                    const T cb = (T)P.anis2 * inv_ms * em * em * em;
                    hx += cb * eux;
                    hy += cb * euy;
                    hz += cb * euz;
                    // cubic, in the principal axes c_i: -2 Kc1 m_i (m_j^2 + m_k^2)
                    // - 2 Kc2 m_i m_j^2 m_k^2, over mu0 Ms, mapped back along c_i
                    T pr[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        pr[a] = (T)P.ec[a][0] * mx + (T)P.ec[a][1] * my + (T)P.ec[a][2] * mz;
                    const T s0 = pr[0] * pr[0], s1 = pr[1] * pr[1], s2 = pr[2] * pr[2];
                    const T c1 = (T)P.cub1 * inv_ms, c2 = (T)P.cub2 * inv_ms;
                    const T g0 = -(c1 * pr[0] * (s1 + s2) + c2 * pr[0] * s1 * s2);
                    const T g1 = -(c1 * pr[1] * (s2 + s0) + c2 * pr[1] * s2 * s0);
                    const T g2 = -(c1 * pr[2] * (s0 + s1) + c2 * pr[2] * s0 * s1);
                    hx += g0 * (T)P.ec[0][0] + g1 * (T)P.ec[1][0] + g2 * (T)P.ec[2][0];
                    hy += g0 * (T)P.ec[0][1] + g1 * (T)P.ec[1][1] + g2 * (T)P.ec[2][1];
                    hz += g0 * (T)P.ec[0][2] + g1 * (T)P.ec[1][2] + g2 * (T)P.ec[2][2];
                }
            }
            if (P.with_oe && h_oe) {
                const T so = (T)P.oe_scale;
                hx += so * elem<true>(h_oe, c0);
                hy += so * elem<true>(h_oe + N, c0);
                hz += so * elem<true>(h_oe + 2 * (size_t)N, c0);
            }
            if (P.with_zee) {
                hx += (T)P.H[0];
                hy += (T)P.H[1];
                hz += (T)P.H[2];
                if (mask && mask[c0]) {
                    hx += (T)P.Hd[0];
                    hy += (T)P.Hd[1];
                    hz += (T)P.Hd[2];
                }
            }
        }
        if (h_out) {
            elem<true>(h_out, c0) = hx;
            elem<true>(h_out + N, c0) = hy;
            elem<true>(h_out + 2 * (size_t)N, c0) = hz;
        }
        // m x h and m x (m x h)
        const T px = my * hz - mz * hy, py = mz * hx - mx * hz, pz = mx * hy - my * hx;
        if (dm_out) {
            const T qx = my * pz - mz * py, qy = mz * px - mx * pz, qz = mx * py - my * px;
            const T gp = (T)P.gp, al = (T)P.alpha, pf = P.precess ? (T)1 : (T)0;
            const bool mag = ms != (T)0;
            const T d[3] = {mag ? -gp * (pf * px + al * qx) : (T)0,
                            mag ? -gp * (pf * py + al * qy) : (T)0,
                            mag ? -gp * (pf * pz + al * qz) : (T)0};
            elem<true>(dm_out, c0) = d[0];
            elem<true>(dm_out + N, c0) = d[1];
            elem<true>(dm_out + 2 * (size_t)N, c0) = d[2];
            if constexpr (ERR) {
                // e = ep + e6 k6 per component, scaled by atol + rtol max(|y|, |y1|)
                const T y1c[3] = {mx, my, mz};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double yv = (double)elem<true>(E.y + (size_t)c * N, c0);
                    if (!isfinite(yv)) ebad += 1.0;
                    if (PERCELL && !mag) continue;
                    const double e =
                        (double)elem<true>(E.ep + (size_t)c * N, c0) + E.e6 * (double)d[c];
                    const double ya = fabs(yv), yb = fabs((double)y1c[c]);
                    const double scl = E.atol + E.rtol * (ya > yb ? ya : yb);
                    const double r = e / scl;
                    eacc += r * r;
                }
            }
        }
        if (torque && ms != (T)0) {
            const double tq = sqrt((double)px * px + (double)py * py + (double)pz * pz) / (double)ms;
            tmax = tmax > tq ? tmax : tq;
        }
    }
    if (torque) {
        // wavefront max, then one atomic per wavefront
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_down(tmax, off, 64);
            tmax = tmax > o ? tmax : o;
        }
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(torque, tmax);
    }
    if constexpr (ERR) {
        // block partials in a fixed order: a wavefront tree, then the
        // wavefronts in order
        __shared__ double esum[2][G::kNT / 64];
        for (int off = 32; off > 0; off >>= 1) {
            eacc += __shfl_down(eacc, off, 64);
            ebad += __shfl_down(ebad, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            esum[0][threadIdx.x >> 6] = eacc;
            esum[1][threadIdx.x >> 6] = ebad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < G::kNT / 64; ++w) {
                s0 += esum[0][w];
                s1 += esum[1][w];
            }
            E.part[lb] = s0;
            E.part[nblocks + lb] = s1;
        }
    }
}

// ---------------------------------------------------------------------------
// Dispatch helpers (power-of-two lengths 1..1024).
// ---------------------------------------------------------------------------
#define MMX_CASES(MACRO) \
    MACRO(1) MACRO(2) MACRO(4) MACRO(8) MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) \
    MACRO(512) MACRO(1024)

template <typename T, int L, int DIR>
static hipError_t launch_strided_L(const Plan& p, const cx<T>* in, cx<T>* out, int n_in, int n_out,
                                   long es_in, long es_out, int ncols, int G1, long g1_in,
                                   long g1_out, int G2, long g2_in, long g2_out)
{
    using G = Strided<T, L>;
    const int ntile = (ncols + G::kB - 1) / G::kB;
    const long nblocks = (long)ntile * G2 * G1;
    const long grid = xcd_grid(nblocks);
    const bool half = DIR < 0 ? 2 * n_in <= L : 2 * n_out <= L;
    // one past the largest element offset touched in `in` / `out`
    const long top_in = (long)(G1 - 1) * g1_in + (long)(G2 - 1) * g2_in + ncols +
                        (long)(n_in > 0 ? n_in - 1 : 0) * es_in;
    const long top_out = (long)(G1 - 1) * g1_out + (long)(G2 - 1) * g2_out + ncols +
                         (long)(n_out > 0 ? n_out - 1 : 0) * es_out;
    const bool o32 = (size_t)std::max(top_in, top_out) * sizeof(cx<T>) < (1ull << 32);
#define MMX_KS(H, O)                                                                              \
    k_strided<T, L, DIR, H, O><<<grid, G::kB * G::kT, 0, p.stream>>>(                             \
        in, out, n_in, n_out, es_in, es_out, ncols, ntile, G2, nblocks, g1_in, g1_out, g2_in,    \
        g2_out, (const cx<T>*)p.tw, p.Lmax)
    if (half && L > 1 && o32)
        MMX_KS(true, true);
    else if (half && L > 1)
        MMX_KS(true, false);
    else if (o32)
        MMX_KS(false, true);
    else
        MMX_KS(false, false);
#undef MMX_KS
    return hipGetLastError();
}

template <typename T, int DIR>
hipError_t launch_strided(const Plan& p, int L, const cx<T>* in, cx<T>* out, int n_in,
                                 int n_out, long es_in, long es_out, int ncols, int G1,
                                 long g1_in, long g1_out, int G2, long g2_in, long g2_out)
{
    switch (L) {
#define MMX_S(LL)                                                                               \
    case LL:                                                                                    \
        return launch_strided_L<T, LL, DIR>(p, in, out, n_in, n_out, es_in, es_out, ncols, G1, \
                                            g1_in, g1_out, G2, g2_in, g2_out);
        MMX_CASES(MMX_S)
#undef MMX_S
    }
    return hipErrorInvalidValue;
}

template <typename T, int M, bool PC>
static hipError_t launch_x_r2c_M(const Plan& p, const T* in, long in_row, long in_comp, int n_in,
                                 const T* Ms_cell, T Ms, cx<T>* out, long out_row, long out_comp,
                                 int nrows, int ncomp, const StageIn<T>* sc);

template <typename T, bool PC>
hipError_t launch_x_r2c(const Plan& p, int M, const T* in, long in_row, long in_comp,
                               int n_in, const T* Ms_cell, T Ms, cx<T>* out, long out_row,
                               long out_comp, int nrows, int ncomp, const StageIn<T>* sc = nullptr)
{
    // a stage input needs the transform kernel (M >= 2) and in == sc->y
    if (sc && (M < 2 || in != sc->y || !sc->ys)) return hipErrorInvalidValue;
    switch (M) {
#define MMX_X(LL)                                                                                 \
    case LL:                                                                                      \
        return launch_x_r2c_M<T, LL, PC>(p, in, in_row, in_comp, n_in, Ms_cell, Ms, out, out_row, \
                                         out_comp, nrows, ncomp, sc);
        MMX_X(0) MMX_CASES(MMX_X)
#undef MMX_X
    }
    return hipErrorInvalidValue;
}

// Px == 1: the x transform of a single cell is the cell value itself.
template <typename T, bool PERCELL>
__global__ void k_x_copy(const T* __restrict__ in, long in_row, long in_comp, int n_in,
                         const T* __restrict__ Ms_cell, T Ms, cx<T>* __restrict__ out, long out_row,
                         long out_comp, int nrows, int ncomp)
{
    const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (long)nrows * ncomp) return;
    const long c = row / nrows, r = row % nrows;
    T a = n_in > 0 ? in[c * in_comp + r * in_row] * (PERCELL ? Ms_cell[r * in_row] : Ms) : (T)0;
    out[c * out_comp + r * out_row] = {a, (T)0};
}

template <typename T, int M, bool PC>
static hipError_t launch_x_r2c_M(const Plan& p, const T* in, long in_row, long in_comp, int n_in,
                                 const T* Ms_cell, T Ms, cx<T>* out, long out_row, long out_comp,
                                 int nrows, int ncomp, const StageIn<T>* sc)
{
    const long rows = (long)nrows * ncomp;
    if constexpr (M == 0 || M == 1) {
        k_x_copy<T, PC><<<(rows + 255) / 256, 256, 0, p.stream>>>(in, in_row, in_comp, n_in, Ms_cell,
                                                                   Ms, out, out_row, out_comp,
                                                                   nrows, ncomp);
    } else {
        using G = XR2C<T, M>;
        const long grid = (rows + G::kRows - 1) / G::kRows;
        const uintptr_t al = 2 * sizeof(T) - 1;
        bool vec = n_in % 2 == 0 && in_row % 2 == 0 && in_comp % 2 == 0 &&
                   ((uintptr_t)in & al) == 0 && (!PC || ((uintptr_t)Ms_cell & al) == 0);
        if (sc) {
            vec = vec && ((uintptr_t)sc->ys & al) == 0 && ((uintptr_t)sc->ep & al) == 0;
            for (int j = 0; j < 7; ++j)
                if (sc->c[j] != 0.0 || (sc->ep && sc->e[j] != 0.0))
                    vec = vec && ((uintptr_t)sc->k[j] & al) == 0;
        }
        const StageIn<T> none{};
        const dim3 blk(G::kRows * G::kT);
#define MMX_XL(HF, CB)                                                                          \
    k_x_r2c<T, M, PC, HF, CB><<<grid, blk, 0, p.stream>>>(in, in_row, in_comp, n_in, Ms_cell, Ms, \
                                                          out, out_row, out_comp, nrows, ncomp, \
                                                          (const cx<T>*)p.tw, p.Lmax, vec,      \
                                                          CB ? *sc : none,                      \
                                                          PC ? nullptr : (const T*)p.Ms_b)
        if (n_in <= M) {
            if (sc) MMX_XL(true, true); else MMX_XL(true, false);
        } else {
            if (sc) MMX_XL(false, true); else MMX_XL(false, false);
        }
#undef MMX_XL
    }
    return hipGetLastError();
}

template <typename T, int L, int AXIS, int PROD = 0>
static hipError_t launch_mid_L(const Plan& p, cx<T>* S, int n_valid, long es, long cs,
                               long gstride, int G)
{
    // AXIS = 2 pairs ky with Py - ky: groups 0 .. Py/2
    const int groups = (AXIS == 2 && G > 1) ? G / 2 + 1 : G;
    const bool o32 = (size_t)p.S2n * 2 * sizeof(T) < (1ull << 32) &&
                     (size_t)p.Kn * 6 * sizeof(T) < (1ull << 32);
    const bool half = 2 * n_valid <= L && L > 1;
    if constexpr (MMX_MIDW && MidW<T, L>::kOK) {
        using Gw = MidW<T, L>;
        const int ntile = (p.Hx + Gw::kCB - 1) / Gw::kCB;
        const int ntb = ntile;
        const long nb = AXIS == 2 ? (long)ntb * groups : (ntile + Gw::kW - 1) / Gw::kW;
        // a batch: the requests' spectra follow each other, 3 components apart
        const int nbatch = p.batch > 1 ? p.batch : 1;
#define MMX_KMIDW(H, O)                                                                           \
    k_mid_w<T, L, AXIS, H, O, PROD><<<xcd_grid(nb * nbatch), 64 * Gw::kW, 0, p.stream>>>(         \
        S, (const T*)p.Khat, n_valid, es, cs, gstride, p.Hx, ntb, nb, p.P[1], p.P[2], p.Kn,       \
        p.Hxp, (const cx<T>*)p.tw, p.Lmax, nbatch, 3 * cs)
        if (half && o32)
            MMX_KMIDW(true, true);
        else if (half)
            MMX_KMIDW(true, false);
        else if (o32)
            MMX_KMIDW(false, true);
        else
            MMX_KMIDW(false, false);
#undef MMX_KMIDW
        return hipGetLastError();
    } else {
    if (p.batch > 1) return hipErrorInvalidValue;  // batches need the wave-local kernel
    using Gm = Mid<T, L>;
    const int ntile = (p.Hx + Gm::kB - 1) / Gm::kB;
    const long nblocks = (long)ntile * groups;
    // the Oersted product (PROD 1) uses the paired-in-block order only
    const bool adj = PROD == 0 && (sizeof(T) == 4 ? MMX_MID_ADJ_F32 : MMX_MID_ADJ_F64) &&
                     AXIS == 2 && G > 1;
    const long nb = adj ? 2 * nblocks : nblocks;
#define MMX_KMID(H, O, AD)                                                                        \
    k_mid<T, L, AXIS, H, O, AD, PROD><<<xcd_grid(nb), Gm::kB * Gm::kT, 0, p.stream>>>(            \
        S, (const T*)p.Khat, n_valid, es, cs, gstride, p.Hx, ntile, nb, p.P[1], p.P[2], p.Kn,     \
        p.Hxp, (const cx<T>*)p.tw, p.Lmax)
#define MMX_KMID2(H, O)                  \
    if constexpr (PROD == 0) {           \
        if (adj)                         \
            MMX_KMID(H, O, true);        \
        else                             \
            MMX_KMID(H, O, false);       \
    } else {                             \
        MMX_KMID(H, O, false);           \
    }
    if (half && o32) {
        MMX_KMID2(true, true)
    } else if (half) {
        MMX_KMID2(true, false)
    } else if (o32) {
        MMX_KMID2(false, true)
    } else {
        MMX_KMID2(false, false)
    }
#undef MMX_KMID2
#undef MMX_KMID
    return hipGetLastError();
    }
}

template <typename T, int AXIS, int PROD = 0>
hipError_t launch_mid(const Plan& p, int L, cx<T>* S, int n_valid, long es, long cs,
                             long gstride, int G)
{
    switch (L) {
#define MMX_M(LL) \
    case LL: return launch_mid_L<T, LL, AXIS, PROD>(p, S, n_valid, es, cs, gstride, G);
        MMX_CASES(MMX_M)
#undef MMX_M
    }
    return hipErrorInvalidValue;
}

// err: also accumulate the error norm's block partials (plain stencil, one
// request, wave-local kernel); *nb_out: the number of blocks (partial pairs).
template <typename T, int M, bool PC, int EXT>
static hipError_t launch_local_M(const Plan& p, const T* m, T* h, T* dm, const LocalParams& P,
                                 double* torque, const LocalErr<T>* err, long* nb_out,
                                 const T* m_lo)
{
    if constexpr (MMX_X1W && XC2RW<T, M>::kOK) {
        using Gw = XC2RW<T, M>;
        const int njt = (p.n[1] + Gw::kRB - 1) / Gw::kRB;
        const long nblocks = (long)njt * p.n[2];
        if (nb_out) *nb_out = nblocks;
        if (m_lo) {
            // the split state (FP32 fields of a double state): plain stencil,
            // one material per request
            if constexpr (std::is_same<T, float>::value && !PC && EXT == 0) {
                if (err || p.layered) return hipErrorInvalidValue;
                if (p.Pb) {
                    k_x_c2r_local_w<T, M, false, EXT_LO, true>
                        <<<xcd_grid(nblocks * p.batch), Gw::kNT, 0, p.stream>>>(
                            (const cx<T>*)p.S1, m, h, dm, nullptr, nullptr, P, torque, nblocks,
                            (const cx<T>*)p.tw, p.Lmax, nullptr, nullptr, nullptr, nullptr,
                            nullptr, (const LocalParams*)p.Pb, p.batch, 8, LocalErr<T>{}, m_lo);
                } else {
                    k_x_c2r_local_w<T, M, false, EXT_LO, false>
                        <<<xcd_grid(nblocks), Gw::kNT, 0, p.stream>>>(
                            (const cx<T>*)p.S1, m, h, dm, nullptr, p.mask, P, torque, nblocks,
                            (const cx<T>*)p.tw, p.Lmax, nullptr, nullptr, nullptr,
                            P.with_oe ? (const T*)p.h_oe : nullptr, nullptr, nullptr, 1, 0,
                            LocalErr<T>{}, m_lo);
                }
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        }
        if (err) {
            if constexpr (EXT == 0) {
                if (p.Pb || !dm || !err->part || nblocks > (long)p.n[1] * p.n[2])
                    return hipErrorInvalidValue;
                k_x_c2r_local_w<T, M, PC, 0, false, true>
                    <<<xcd_grid(nblocks), Gw::kNT, 0, p.stream>>>(
                        (const cx<T>*)p.S1, m, h, dm, (const T*)p.Ms_cell, p.mask, P, torque,
                        nblocks, (const cx<T>*)p.tw, p.Lmax, nullptr, nullptr,
                        p.layered ? (const T*)p.zw : nullptr, P.with_oe ? (const T*)p.h_oe : nullptr,
                        nullptr, nullptr, 1, 0, *err, nullptr);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        }
        if (p.Pb) {
            // a batch plan: uniform material per request, constants from
            // p.Pb, p.batch requests per launch, torque maxima 8 doubles apart
            if constexpr (!PC && EXT == 0) {
                if (p.layered || p.batch < 1) return hipErrorInvalidValue;
                k_x_c2r_local_w<T, M, false, 0, true>
                    <<<xcd_grid(nblocks * p.batch), Gw::kNT, 0, p.stream>>>(
                        (const cx<T>*)p.S1, m, h, dm, nullptr, nullptr, P, torque, nblocks,
                        (const cx<T>*)p.tw, p.Lmax, nullptr, nullptr, nullptr, nullptr, nullptr,
                        (const LocalParams*)p.Pb, p.batch, 8, LocalErr<T>{}, nullptr);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        }
        k_x_c2r_local_w<T, M, PC, EXT, false><<<xcd_grid(nblocks), Gw::kNT, 0, p.stream>>>(
            (const cx<T>*)p.S1, m, h, dm, (const T*)p.Ms_cell, p.mask, P, torque, nblocks,
            (const cx<T>*)p.tw, p.Lmax, (EXT & EXT_PA) ? (const T*)p.A_cell : nullptr,
            (EXT & EXT_PD) ? (const T*)p.D_cell : nullptr, p.layered ? (const T*)p.zw : nullptr,
            P.with_oe ? (const T*)p.h_oe : nullptr,
            EXT != 0 && p.percell_Ku ? (const T*)p.Ku_cell : nullptr, nullptr, 1, 0,
            LocalErr<T>{}, nullptr);
        return hipGetLastError();
    }
    // batches, the error accumulation and the split state need the
    // wave-local kernel
    if (p.Pb || err || m_lo) return hipErrorInvalidValue;
    if (nb_out) *nb_out = 0;
    using G = XC2R<T, M>;
    const int njt = (p.n[1] + G::kRows - 1) / G::kRows;
    const long nblocks = (long)njt * p.n[2];
    k_x_c2r_local<T, M, PC, EXT><<<xcd_grid(nblocks), G::kRows * 3 * G::kT, 0, p.stream>>>(
        (const cx<T>*)p.S1, m, h, dm, (const T*)p.Ms_cell, p.mask, P, torque, njt, nblocks,
        (const cx<T>*)p.tw, p.Lmax, (EXT & EXT_PA) ? (const T*)p.A_cell : nullptr,
        (EXT & EXT_PD) ? (const T*)p.D_cell : nullptr, p.layered ? (const T*)p.zw : nullptr,
        P.with_oe ? (const T*)p.h_oe : nullptr,
        EXT != 0 && p.percell_Ku ? (const T*)p.Ku_cell : nullptr);
    return hipGetLastError();
}

template <typename T, bool PC, int EXT>
hipError_t launch_local(const Plan& p, int M, const T* m, T* h, T* dm,
                               const LocalParams& P, double* torque,
                               const LocalErr<T>* err = nullptr, long* nb_out = nullptr,
                               const T* m_lo = nullptr)
{
    switch (M) {
#define MMX_L(LL) \
    case LL: return launch_local_M<T, LL, PC, EXT>(p, m, h, dm, P, torque, err, nb_out, m_lo);
        MMX_L(0) MMX_CASES(MMX_L)
#undef MMX_L
    }
    return hipErrorInvalidValue;
}


// The local pass in an extended stencil variant (ext != 0: DMI, per-cell A,
// per-cell D, mixed-sign D, per-cell Ku), dispatched at run time; explicitly
// instantiated per precision in its own translation unit (local_ext_*.hip).
template <typename T>
hipError_t launch_local_ext(const Plan& p, int M, const T* m, T* h, T* dm, const LocalParams& P,
                            double* torque, bool pc, int ext)
{
    switch (ext) {
#define MMX_X(E)                                                              \
    case E:                                                                   \
        return pc ? launch_local<T, true, E>(p, M, m, h, dm, P, torque)       \
                  : launch_local<T, false, E>(p, M, m, h, dm, P, torque);
        MMX_X(EXT_DMI)
        MMX_X(EXT_PA)
        MMX_X(EXT_DMI | EXT_PA)
        MMX_X(EXT_DMI | EXT_PD)
        MMX_X(EXT_DMI | EXT_PA | EXT_PD)
        MMX_X(EXT_DMI | EXT_PD | EXT_MIX)
        MMX_X(EXT_DMI | EXT_PA | EXT_PD | EXT_MIX)
        MMX_X(EXT_PK)
#undef MMX_X
    }
    return hipErrorInvalidValue;
}

// Explicit instantiations of the pass launchers, one translation unit per
// precision (passes_f32.hip / passes_f64.hip); the rest of the pipeline sees
// them as extern templates.
#define MMX_PASS_INST(EXT_, T)                                                                   \
    EXT_ template hipError_t launch_strided<T, -1>(const Plan&, int, const cx<T>*, cx<T>*, int, \
                                                   int, long, long, int, int, long, long, int,  \
                                                   long, long);                                 \
    EXT_ template hipError_t launch_strided<T, 1>(const Plan&, int, const cx<T>*, cx<T>*, int,  \
                                                  int, long, long, int, int, long, long, int,   \
                                                  long, long);                                  \
    EXT_ template hipError_t launch_x_r2c<T, false>(const Plan&, int, const T*, long, long, int, \
                                                    const T*, T, cx<T>*, long, long, int, int,  \
                                                    const StageIn<T>*);                         \
    EXT_ template hipError_t launch_x_r2c<T, true>(const Plan&, int, const T*, long, long, int,  \
                                                   const T*, T, cx<T>*, long, long, int, int,   \
                                                   const StageIn<T>*);                          \
    EXT_ template hipError_t launch_local<T, false, 0>(const Plan&, int, const T*, T*, T*,      \
                                                       const LocalParams&, double*,             \
                                                       const LocalErr<T>*, long*, const T*);    \
    EXT_ template hipError_t launch_local<T, true, 0>(const Plan&, int, const T*, T*, T*,       \
                                                      const LocalParams&, double*,              \
                                                      const LocalErr<T>*, long*, const T*);
#define MMX_MID_INST(EXT_, T)                                                                    \
    EXT_ template hipError_t launch_mid<T, 2, 0>(const Plan&, int, cx<T>*, int, long, long,     \
                                                 long, int);                                    \
    EXT_ template hipError_t launch_mid<T, 1, 0>(const Plan&, int, cx<T>*, int, long, long,     \
                                                 long, int);                                    \
    EXT_ template hipError_t launch_mid<T, 2, 1>(const Plan&, int, cx<T>*, int, long, long,     \
                                                 long, int);                                    \
    EXT_ template hipError_t launch_mid<T, 1, 1>(const Plan&, int, cx<T>*, int, long, long,     \
                                                 long, int);

}  // namespace mmx
