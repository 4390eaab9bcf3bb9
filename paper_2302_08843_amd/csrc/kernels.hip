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
template <typename T, int M>
struct XR2C {
    using S = FFTShape<M, Regs<T>::x>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kRows = cmax(1, MMX_XBLOCK / kT);
};

template <typename T, int M, bool PERCELL, bool HALF>
__global__ __launch_bounds__((XR2C<T, M>::kRows * XR2C<T, M>::kT)) void k_x_r2c(
    const T* __restrict__ in, long in_row, long in_comp, int n_in, const T* __restrict__ Ms_cell,
    T Ms, cx<T>* __restrict__ out, long out_row, long out_comp, int nrows, int ncomp,
    const cx<T>* __restrict__ tw, int Lmax, bool vec)
{
    using G = XR2C<T, M>;
    constexpr int kE = G::kE, kT = G::kT, kRows = G::kRows;
    constexpr int kL = G::S::kLds;  // LDS slots per row
    __shared__ cx<T> lds[kRows * kL];
    const int t = threadIdx.x % kT, rl = threadIdx.x / kT;
    const long row = (long)blockIdx.x * kRows + rl;
    const bool valid = row < (long)nrows * ncomp;
    const long c = valid ? row / nrows : 0, r = valid ? row % nrows : 0;
    const T* src = in + c * in_comp + r * in_row;
    const T* msrc = PERCELL ? Ms_cell + r * in_row : nullptr;
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
                if (valid && i0 < n_in) a = src[i0] * (PERCELL ? msrc[i0] : Ms);
                if (valid && i1 < n_in) b = src[i1] * (PERCELL ? msrc[i1] : Ms);
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
__global__ __launch_bounds__((Strided<T, L>::kB * Strided<T, L>::kT)) void k_strided(
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
    using S = FFTShape<L, Regs<T>::mid>;
    static constexpr int kE = S::kE, kT = S::kT;
    static constexpr int kB =
        cmin(64, cmax(1, (sizeof(T) == 4 ? MMX_MBLOCK : MMX_MBLOCK_F64) / kT));
};

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

// One pencil group (fixed ky for AXIS = 2) of the last-axis pass: load three
// components, forward transform, product with the spectral kernel, inverse
// transform, store.  HALF: n_valid <= L/2 (always true with zero padding).
// Element (c, e) of the group is S[o + c*cs + e*es]; index arithmetic is done
// in 32 bits when O32.  PROD 0: the symmetric demag product with the six
// folded real components; PROD 1: the Oersted product h = j x (i g) with the
// three folded components g (imaginary spectrum, odd along its own axis).
template <typename T, int L, int AXIS, bool HALF, bool O32, int PROD = 0>
__device__ __forceinline__ void mid_group(cx<T>* S, long o_, const T* __restrict__ Khat,
                                          int n_valid, long es_, long cs_, bool cv, int col, int g,
                                          int t, int b, cx<T>* lds, int Py, int Pz, long Kn_,
                                          int Hxp, const cx<T>* __restrict__ tw, int Lmax)
{
    using I = typename std::conditional<O32, unsigned, long>::type;
    using G = Mid<T, L>;
    constexpr int kE = G::kE, kT = G::kT, kB = G::kB;
    const I o = (I)o_, es = (I)es_, cs = (I)cs_, Kn = (I)Kn_;
    cx<T> v[3][kE];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < kE; ++r) {
            const int e = t + r * kT;
            v[c][r] = (!(HALF && r >= kE / 2) && cv && e < n_valid)
                          ? elem<O32>((const cx<T>*)S, o + (I)c * cs + (I)e * es)
                          : cx<T>{0, 0};
        }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        WgFFT<T, L, Regs<T>::mid, -1, HALF>::run(v[c], t, lds + b, kB, tw, Lmax / L);

    if (cv) {
        const int hy = Py / 2, hz = Pz / 2;
        const I plane = (I)(hy + 1) * (I)Hxp;
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
            const I kb = (I)kzf * plane + (I)kyf * (I)Hxp + (I)col;
            if constexpr (PROD == 1) {
                const T gx = elem<O32>(Khat, kb), gy = sy * elem<O32>(Khat, kb + Kn);
                const T gz = sz * elem<O32>(Khat, kb + 2 * Kn);
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
            const T kxx = elem<O32>(Khat, kb), kyy = elem<O32>(Khat, kb + Kn);
            const T kzz = elem<O32>(Khat, kb + 2 * Kn);
            const T kxy = sy * elem<O32>(Khat, kb + 3 * Kn), kxz = sz * elem<O32>(Khat, kb + 4 * Kn);
            const T kyz = sy * sz * elem<O32>(Khat, kb + 5 * Kn);
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
        WgFFT<T, L, Regs<T>::mid, 1>::run(v[c], t, lds + b, kB, tw, Lmax / L);
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
    mid_group<T, L, AXIS, HALF, O32, PROD>(S, (long)g * gstride + col, Khat, n_valid, es, cs, cv,
                                           col, g, t, b, lds, Py, Pz, Kn, Hxp, tw, Lmax);
    if (paired) {
        const int g2 = Py - g;
        mid_group<T, L, AXIS, HALF, O32, PROD>(S, (long)g2 * gstride + col, Khat, n_valid, es, cs,
                                               cv, col, g2, t, b, lds, Py, Pz, Kn, Hxp, tw, Lmax);
    }
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
static hipError_t launch_strided(const Plan& p, int L, const cx<T>* in, cx<T>* out, int n_in,
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
                                 int nrows, int ncomp);

template <typename T, bool PC>
static hipError_t launch_x_r2c(const Plan& p, int M, const T* in, long in_row, long in_comp,
                               int n_in, const T* Ms_cell, T Ms, cx<T>* out, long out_row,
                               long out_comp, int nrows, int ncomp)
{
    switch (M) {
#define MMX_X(LL)                                                                                 \
    case LL:                                                                                      \
        return launch_x_r2c_M<T, LL, PC>(p, in, in_row, in_comp, n_in, Ms_cell, Ms, out, out_row, \
                                         out_comp, nrows, ncomp);
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
                                 int nrows, int ncomp)
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
        const bool vec = n_in % 2 == 0 && in_row % 2 == 0 && in_comp % 2 == 0 &&
                         ((uintptr_t)in & al) == 0 && (!PC || ((uintptr_t)Ms_cell & al) == 0);
        if (n_in <= M)
            k_x_r2c<T, M, PC, true><<<grid, G::kRows * G::kT, 0, p.stream>>>(
                in, in_row, in_comp, n_in, Ms_cell, Ms, out, out_row, out_comp, nrows, ncomp,
                (const cx<T>*)p.tw, p.Lmax, vec);
        else
            k_x_r2c<T, M, PC, false><<<grid, G::kRows * G::kT, 0, p.stream>>>(
                in, in_row, in_comp, n_in, Ms_cell, Ms, out, out_row, out_comp, nrows, ncomp,
                (const cx<T>*)p.tw, p.Lmax, vec);
    }
    return hipGetLastError();
}

template <typename T, int L, int AXIS, int PROD = 0>
static hipError_t launch_mid_L(const Plan& p, cx<T>* S, int n_valid, long es, long cs,
                               long gstride, int G)
{
    // AXIS = 2 pairs ky with Py - ky: groups 0 .. Py/2
    const int groups = (AXIS == 2 && G > 1) ? G / 2 + 1 : G;
    using Gm = Mid<T, L>;
    const int ntile = (p.Hx + Gm::kB - 1) / Gm::kB;
    const long nblocks = (long)ntile * groups;
    const bool o32 = (size_t)p.S2n * 2 * sizeof(T) < (1ull << 32) &&
                     (size_t)p.Kn * 6 * sizeof(T) < (1ull << 32);
    const bool half = 2 * n_valid <= L && L > 1;
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

template <typename T, int AXIS, int PROD = 0>
static hipError_t launch_mid(const Plan& p, int L, cx<T>* S, int n_valid, long es, long cs,
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

template <typename T, int M, bool PC, int EXT>
static hipError_t launch_local_M(const Plan& p, const T* m, T* h, T* dm, const LocalParams& P,
                                 double* torque)
{
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
static hipError_t launch_local(const Plan& p, int M, const T* m, T* h, T* dm,
                               const LocalParams& P, double* torque)
{
    switch (M) {
#define MMX_L(LL) \
    case LL: return launch_local_M<T, LL, PC, EXT>(p, m, h, dm, P, torque);
        MMX_L(0) MMX_CASES(MMX_L)
#undef MMX_L
    }
    return hipErrorInvalidValue;
}

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

__global__ void k_fill(double* p, int n, double v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Coefficients of a stage combination.  h: if not null, every coefficient is
// multiplied by *h (the step size held on the device by the device-side
// controller); the host-driven path folds h into c and leaves h null.
struct Coef7 {
    double c[7];
    const double* h;
};

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
    const double hs = cf.h ? *cf.h : 1.0;
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
    const double hs = cf.h ? *cf.h : 1.0;
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
__global__ void k_dp_begin(DevCtl* c)
{
    if (c->done) return;
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

__global__ void k_dp_control(DevCtl* c, const double* __restrict__ red)
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

__global__ void k_dp_torque(DevCtl* c, const double* __restrict__ red)
{
    if (!c->done) c->torque = red[1];
}

// y = y1 (renormalised on magnetic cells, zero on vacuum cells, when
// c->renorm) and k0 = k6 (without renorm), on acceptance only.
template <typename T>
__global__ void k_dp_commit(const DevCtl* __restrict__ c, T* __restrict__ y,
                            const T* __restrict__ y1, T* __restrict__ k0,
                            const T* __restrict__ k6, const T* __restrict__ Ms_cell, long N)
{
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
    q.tw = tw64;
    const long hyx = (long)(Py / 2 + 1) * p.Hxp;
    for (int comp = 0; comp < 6; ++comp)
        for (int t = 0; t < nz; ++t)
            for (int s = 0; s < nz; ++s) {
                k_place_layer<<<blocks_for(PN, 256), 256, 0, p.stream>>>(
                    R, comp, t, s, nx, ny, nz, Px, Py, near, nI, nJ, zb, p.demag_p, p.d[0], p.d[1]);
                MMX_TRY(hipGetLastError());
                MMX_TRY((launch_x_r2c<double, false>(q, Px / 2, R, Px, 0, Px, nullptr, 1.0, C,
                                                     p.Hxp, 0, Py, 1)));
                if (Py > 1)
                    MMX_TRY((launch_strided<double, -1>(q, Py, C, C, Py, Py, p.Hxp, p.Hxp, p.Hx, 1,
                                                        0, 0, 1, 0, 0)));
                k_fold_layer<T><<<blocks_for(hyx, 256), 256, 0, p.stream>>>(
                    (T*)p.Khat + comp * p.Kn + ((long)t * nz + s) * hyx, C, p.Hx, p.Hxp, Py,
                    comp >= 4 ? 1 : 0, 1.0 / (double)PN);
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
//   h^_t(kx, ky) = sum_s K^^{ts}(kx, ky) M^_s(kx, ky),
// in place on the y-transformed spectrum S ([3][nz][Py][Hxp]).  K^ is
// [6][nz][nz][Py/2+1][Hxp]: xx, yy, zz, xy real, xz, yz imaginary (stored as
// their imaginary part); row Py - ky uses row ky with the y-odd components
// (xy, yz) negated.  A block holds TW consecutive kx of the row pair (ky,
// Py - ky), so every kernel row is read once for both: the spectra of all
// layers of both rows are staged in LDS, then thread (kx, g) accumulates
// targets t = g, g + G, ... .
// ---------------------------------------------------------------------------
constexpr int kZdMaxLayers = 16;

template <typename T>
struct ZdTile {
    static constexpr int kTW = sizeof(T) == 4 ? 64 : 32;  // kx per block
};

template <typename T>
__global__ __launch_bounds__(ZdTile<T>::kTW * kZdMaxLayers) void k_zdense(
    cx<T>* __restrict__ S, const T* __restrict__ K, int nz, int Py, int Hx, int Hxp, long s_comp,
    long k_comp)
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
            const long kb = (((long)t * nz + sidx) * hy + ky) * Hxp + kx;
            const T kxx = K[kb], kyy = K[k_comp + kb], kzz = K[2 * k_comp + kb];
            const T kxy = K[3 * k_comp + kb], vxz = K[4 * k_comp + kb], vyz = K[5 * k_comp + kb];
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
                                                 (long)nz * Py * p.Hxp, p.Kn);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Field evaluation.
// ---------------------------------------------------------------------------
// Demag convolution up to the x spectrum: S1 <- spectrum of K (Ms src) (or of
// K src with use_ms = false), i.e. every pass but the last inverse x
// transform, which the caller fuses with its local terms.
template <typename T>
static hipError_t demag_to_S1(Plan& p, const T* m, bool use_ms)
{
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int Py = p.P[1], Pz = p.P[2];
    const int M = p.P[0] / 2;
    const long s1c = (long)nz * ny * p.Hxp;
    cx<T>* S1 = (cx<T>*)p.S1;
    cx<T>* S2 = (cx<T>*)p.S2;
    const bool pc = p.percell && use_ms;
    const T ms = use_ms ? (T)p.Ms : (T)1;
    MMX_TRY(timed(p, MM_PASS_X_FWD, [&] {
        return pc ? launch_x_r2c<T, true>(p, M, m, nx, p.N, nx, (const T*)p.Ms_cell, ms, S1, p.Hxp,
                                          s1c, ny * nz, 3)
                  : launch_x_r2c<T, false>(p, M, m, nx, p.N, nx, nullptr, ms, S1, p.Hxp, s1c,
                                           ny * nz, 3);
    }));
    if (p.layered) {
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
                return launch_strided<T, -1>(p, Py, S1, S2, ny, Py, p.Hxp, p.Hxp, p.Hx, 3, s1c, s2c,
                                             nz, (long)ny * p.Hxp, (long)Py * p.Hxp);
            }));
        MMX_TRY(timed(p, MM_PASS_MID, [&] {
            return launch_mid<T, 2>(p, Pz, S2, nz, (long)Py * p.Hxp, s2c, p.Hxp, Py);
        }));
        if (Py > 1)
            MMX_TRY(timed(p, MM_PASS_Y_INV, [&] {
                return launch_strided<T, 1>(p, Py, S2, S1, Py, ny, p.Hxp, p.Hxp, p.Hx, 3, s2c, s1c,
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

template <typename T>
hipError_t eval_field(Plan& p, const T* m, const double hext[3], unsigned terms, double t,
                      T* h_out, T* dm_out, double alpha_eff, bool precess, double* torque)
{
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int Px = p.P[0], Py = p.P[1], Pz = p.P[2];
    const int M = Px / 2;
    const long s1c = (long)nz * ny * p.Hxp;
    cx<T>* S1 = (cx<T>*)p.S1;
    cx<T>* S2 = (cx<T>*)p.S2;
    const bool pc = p.percell;
    if (terms & MM_DEMAG) MMX_TRY(demag_to_S1<T>(p, m, true));
    LocalParams P;
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    P.N = p.N;
    P.s1_comp = s1c;
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
    if (torque) {
        k_fill<<<1, 64, 0, p.stream>>>(torque, 1, 0.0);
        MMX_TRY(hipGetLastError());
    }
    // DMI and the coupling averages only in the variants that need them
    return timed(p, MM_PASS_X_INV_LOCAL, [&] {
        switch (ext) {
#define MMX_X(E)                                                                  \
    case E:                                                                       \
        return pc ? launch_local<T, true, E>(p, M, m, h_out, dm_out, P, torque)   \
                  : launch_local<T, false, E>(p, M, m, h_out, dm_out, P, torque);
            MMX_X(0)
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
    });
}

// ---------------------------------------------------------------------------
// Runge-Kutta helpers.
// ---------------------------------------------------------------------------
static bool aligned16(const void* q) { return ((uintptr_t)q & 15) == 0; }

template <typename T, int NK>
static hipError_t launch_combine(Plan& p, T* y_out, const T* y, const Coef7& cf, const Ptr7<T>& ks,
                                 bool vec)
{
    const long n3 = 3 * p.N;
    const long work = vec ? n3 / V16<T>::n : n3;
    const int blocks = (int)std::min<long>(blocks_for(work, 256), 8192);
    if (vec)
        k_rk_combine<T, NK, true><<<blocks, 256, 0, p.stream>>>(y_out, y, cf, ks, n3);
    else
        k_rk_combine<T, NK, false><<<blocks, 256, 0, p.stream>>>(y_out, y, cf, ks, n3);
    return hipGetLastError();
}

template <typename T>
hipError_t rk_combine(Plan& p, T* y_out, const T* y, double h, const double* a, T* const* k, int nk,
                      const double* hdev)
{
    Coef7 cf{};
    Ptr7<T> ks{};
    cf.h = hdev;
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
                         int nk, double rtol, double atol, double* out_dev, const double* hdev)
{
    Coef7 cf{};
    Ptr7<T> ks{};
    cf.h = hdev;
    bool vec = (p.N % V16<T>::n) == 0 && aligned16(y) && aligned16(y1) &&
               (!p.percell || aligned16(p.Ms_cell));
    for (int j = 0; j < 7; ++j) {
        cf.c[j] = j < nk ? (hdev ? e[j] : h * e[j]) : 0.0;
        ks.p[j] = j < nk ? k[j] : y;
        vec = vec && aligned16(ks.p[j]);
    }
    const T* msc = p.percell ? (const T*)p.Ms_cell : nullptr;
    // a streaming reduction: about 16 (vector) elements per thread, up to
    // kErrBlocks blocks, so large grids keep 8 waves per SIMD resident and
    // small ones launch few blocks (partials: sums in [0, nb), non-finite
    // counts in [nb, 2 nb)); nb depends on the grid only
    const long nv = 3 * p.N / (vec ? V16<T>::n : 1);
    const int nb = (int)std::max<long>(1, std::min<long>(kErrBlocks, blocks_for(nv, kBlock * 16)));
    MMX_TRY(timed(p, MM_PASS_RK, [&] {
        if (vec && p.percell)
            k_err_norm<T, true, true><<<nb, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol,
                                                                   atol, p.red);
        else if (vec)
            k_err_norm<T, true, false><<<nb, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol,
                                                                    atol, p.red);
        else if (p.percell)
            k_err_norm<T, false, true><<<nb, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol,
                                                                    atol, p.red);
        else
            k_err_norm<T, false, false><<<nb, kBlock, 0, p.stream>>>(y, y1, cf, ks, p.N, msc, rtol,
                                                                     atol, p.red);
        return hipGetLastError();
    }));
    const double cnt = 3.0 * (double)p.n_magnetic;
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red, nb, out_dev, 0, cnt > 0 ? 1.0 / cnt : 0.0, 1);
    MMX_TRY(hipGetLastError());
    // out_dev[5]: number of non-finite entries of the current state y
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red + nb, nb, out_dev, 5, 1.0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t renormalise(Plan& p, T* m)
{
    const int blocks = (int)std::min<long>(blocks_for(p.N, 256), 4096);
    k_renorm<T><<<blocks, 256, 0, p.stream>>>(m, p.percell ? (const T*)p.Ms_cell : nullptr, p.N);
    return hipGetLastError();
}

hipError_t dp_begin(Plan& p, DevCtl* c)
{
    k_dp_begin<<<1, 1, 0, p.stream>>>(c);
    return hipGetLastError();
}

hipError_t dp_control(Plan& p, DevCtl* c)
{
    k_dp_control<<<1, 1, 0, p.stream>>>(c, p.red_out);
    return hipGetLastError();
}

hipError_t dp_torque(Plan& p, DevCtl* c)
{
    k_dp_torque<<<1, 1, 0, p.stream>>>(c, p.red_out);
    return hipGetLastError();
}

template <typename T>
hipError_t dp_commit(Plan& p, DevCtl* c, T* y, const T* y1, T* k0, const T* k6)
{
    const int blocks = (int)std::min<long>(blocks_for(p.N, 256), 4096);
    k_dp_commit<T><<<blocks, 256, 0, p.stream>>>(c, y, y1, k0, k6,
                                                 p.percell ? (const T*)p.Ms_cell : nullptr, p.N);
    return hipGetLastError();
}

template <typename T>
hipError_t anis_energy(Plan& p, const T* m, double* out_dev)
{
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
        m, p.percell ? (const T*)p.Ms_cell : nullptr, p.Ms, p.N, A, p.red,
        p.layered ? p.lw : nullptr, (long)p.n[0] * p.n[1],
        p.percell_Ku ? (const T*)p.Ku_cell : nullptr);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red, kRedBlocks, out_dev, 0, 1.0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t dot_ms(Plan& p, const T* a, const T* b, double* out_dev)
{
    k_dot_ms<T><<<kRedBlocks, kBlock, 0, p.stream>>>(a, b, p.percell ? (const T*)p.Ms_cell : nullptr,
                                                     p.Ms, p.N, p.red, p.layered ? p.lw : nullptr,
                                                     (long)p.n[0] * p.n[1]);
    MMX_TRY(hipGetLastError());
    k_final_sum<<<1, kBlock, 0, p.stream>>>(p.red, kRedBlocks, out_dev, 0, 1.0, 0);
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
                                      double, bool, double*);                                    \
    template hipError_t rk_combine<T>(Plan&, T*, const T*, double, const double*, T* const*,     \
                                      int, const double*);                                       \
    template hipError_t rk_error_norm<T>(Plan&, const T*, const T*, double, const double*,       \
                                         T* const*, int, double, double, double*, const double*); \
    template hipError_t dp_commit<T>(Plan&, DevCtl*, T*, const T*, T*, const T*);                \
    template hipError_t renormalise<T>(Plan&, T*);                                               \
    template hipError_t dot_ms<T>(Plan&, const T*, const T*, double*);                           \
    template hipError_t anis_energy<T>(Plan&, const T*, double*);                                \
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
