// fft.h -- workgroup-cooperative power-of-two FFTs for gfx950.
//
// A transform of length L is held by L/E threads with E complex values each
// in registers.  It runs as a Stockham autosort sequence of radix-R stages
// (R <= E, product of the radices = L): every thread performs E/R butterflies
// per stage, exchanging data through LDS between stages only.  The first stage
// takes its inputs straight from the caller's registers (loaded from global
// memory) and the last stage leaves natural-order outputs in registers, so a
// length-L transform with E*E >= L costs exactly one LDS round trip.
//
// Thread t of a transform owns, on entry, the inputs
//     x[t + r*(L/E)],          r = 0..E-1
// and on exit the outputs
//     X[t + q*T + r*(L/Rl)],   q = 0..E/Rl-1, r = 0..Rl-1   (T = L/E)
// in v[q*Rl + r], where Rl is the last radix (outIndex() below).
//
// Twiddle factors come from a table of Lmax roots of unity w^n =
// exp(-2 pi i n / Lmax) rounded from double (mm_twiddles), indexed with the
// stride Lmax/L.  The small in-register DFTs use compile-time constants.
#pragma once
#include <hip/hip_runtime.h>

namespace mmx {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// cos(2 pi k / 64), k = 0..63 (exact values rounded to 21 digits).
__device__ constexpr double kCos64[64] = {
    1.0, 0.995184726672196886245, 0.980785280403230449126, 0.956940335732208864936,
    0.923879532511286756128, 0.881921264348355029713, 0.831469612302545237079,
    0.773010453362736960811, 0.707106781186547524401, 0.634393284163645498215,
    0.555570233019602224743, 0.471396736825997648556, 0.382683432365089771728,
    0.290284677254462367636, 0.195090322016128267848, 0.0980171403295606019942, 0.0,
    -0.0980171403295606019942, -0.195090322016128267848, -0.290284677254462367636,
    -0.382683432365089771728, -0.471396736825997648556, -0.555570233019602224743,
    -0.634393284163645498215, -0.707106781186547524401, -0.773010453362736960811,
    -0.831469612302545237079, -0.881921264348355029713, -0.923879532511286756128,
    -0.956940335732208864936, -0.980785280403230449126, -0.995184726672196886245, -1.0,
    -0.995184726672196886245, -0.980785280403230449126, -0.956940335732208864936,
    -0.923879532511286756128, -0.881921264348355029713, -0.831469612302545237079,
    -0.773010453362736960811, -0.707106781186547524401, -0.634393284163645498215,
    -0.555570233019602224743, -0.471396736825997648556, -0.382683432365089771728,
    -0.290284677254462367636, -0.195090322016128267848, -0.0980171403295606019942, 0.0,
    0.0980171403295606019942, 0.195090322016128267848, 0.290284677254462367636,
    0.382683432365089771728, 0.471396736825997648556, 0.555570233019602224743,
    0.634393284163645498215, 0.707106781186547524401, 0.773010453362736960811,
    0.831469612302545237079, 0.881921264348355029713, 0.923879532511286756128,
    0.956940335732208864936, 0.980785280403230449126, 0.995184726672196886245};

// v * exp(DIR * 2 pi i k / 64), DIR = -1 forward, +1 inverse.  k is a
// compile-time constant after unrolling; the trivial angles avoid multiplies.
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot64(cx<T> v, int k)
{
    k &= 63;
    if (k == 0) return v;
    if (k == 16) return DIR < 0 ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
    if (k == 32) return {-v.x, -v.y};
    if (k == 48) return DIR < 0 ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
    const T c = (T)kCos64[k];
    const T s = (T)DIR * (T)kCos64[(16 - k) & 63];  // DIR * sin(2 pi k/64)
    return {v.x * c - v.y * s, v.x * s + v.y * c};
}

// Ordering point between the LDS writes and reads of one exchange.  WAVE:
// every thread of the transform lives in the calling wavefront, whose LDS
// instructions execute in issue order, so only the compiler must be kept from
// moving accesses across (wavefront-scope fences, no s_barrier); otherwise a
// workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void fft_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int v, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register DFT of length R <= 64 on a[0..R), natural order in and out.
// Radix-2 decimation in frequency followed by a compile-time bit-reversal
// permutation (register renaming only).  HALF_IN: a[R/2..R) are known to be
// zero (zero padding), so the first butterfly level only rotates.
template <int R, int DIR, bool HALF_IN = false, typename T>
__device__ __forceinline__ void dft(cx<T>* a)
{
    if constexpr (R == 1) {
        return;
    } else {
#pragma unroll
        for (int len = R; len >= 2; len >>= 1) {
            const int half = len >> 1;
#pragma unroll
            for (int s = 0; s < R; s += len) {
#pragma unroll
                for (int k = 0; k < half; ++k) {
                    if (HALF_IN && len == R) {
                        a[s + k + half] = rot64<DIR>(a[s + k], k * (64 / len));
                    } else {
                        cx<T> u = a[s + k], w = a[s + k + half];
                        a[s + k] = cadd(u, w);
                        a[s + k + half] = rot64<DIR>(csub(u, w), k * (64 / len));
                    }
                }
            }
        }
        cx<T> b[R];
#pragma unroll
        for (int k = 0; k < R; ++k) b[k] = a[bitrev(k, ilog2(R))];
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = b[k];
    }
}

// Radix of stage s for a length-L transform with E registers per thread.
constexpr int stage_radix(int L, int E, int s)
{
    int rem = L, r = 1;
    for (int i = 0; i <= s; ++i) {
        r = rem < E ? rem : E;
        rem /= r;
    }
    return r;
}
constexpr int stage_count(int L, int E)
{
    int n = 0;
    for (int rem = L; rem > 1; ++n) rem /= (rem < E ? rem : E);
    return n;
}
constexpr int stage_ns(int L, int E, int s)  // product of radices before stage s
{
    int p = 1;
    for (int i = 0; i < s; ++i) p *= stage_radix(L, E, i);
    return p;
}

template <int L, int E>
struct FFTShape {
    static constexpr int kE = (E < L ? E : L);
    static constexpr int kT = L / kE;                 // threads per transform
    static constexpr int kStages = stage_count(L, kE);
    static constexpr int kLast = kStages > 0 ? stage_radix(L, kE, kStages - 1) : 1;
    // LDS slots per transform: one pad slot after every kE elements.  The
    // first stage writes element j*kE + r from thread j; without the pad all
    // threads of a lane group would hit the same LDS bank.
    static constexpr int kPadLog = ilog2(kE);
    static constexpr int kLds = L + (L >> kPadLog);
    __device__ static constexpr int lds_slot(int e) { return e + (e >> kPadLog); }
    // natural output index held in v[i] after run()
    __device__ static constexpr int out_index(int t, int i)
    {
        return L == 1 ? 0 : t + (i / kLast) * kT + (i % kLast) * (L / kLast);
    }
    // natural input index expected in v[r] before run()
    __device__ static constexpr int in_index(int t, int r) { return t + r * kT; }
};

// One Stockham transform per group of kT threads.  `lds` points to this
// transform's scratch of S::kLds complex slots, slot s at lds[s * lstride].
// All threads of the workgroup (WAVE: of the wavefront, which then holds the
// whole transform) must call run(), also those whose transform is masked out.  HALF_IN: the inputs x[L/2..L) are zero
// (the caller leaves v[kE/2..kE) zero; the first stage skips them).
// SPLIT: the scratch holds S::kLds reals (slot s at ((T*)lds)[s * lstride])
// and every exchange moves the real parts, then the imaginary parts -- half
// the LDS per transform for two more barriers per exchange.
template <typename T, int L, int E, int DIR, bool HALF_IN = false, bool SPLIT = false,
          bool WAVE = false>
struct WgFFT {
    using S = FFTShape<L, E>;
    static constexpr int kE = S::kE;
    static constexpr int kT = S::kT;

    // Exchange after stage s: element base_j + r*Ns of butterfly j written by
    // stage s, element j + r*(L/R') read for stage s+1 (radix R'), one real
    // half at a time.
    template <int s>
    __device__ static __forceinline__ void split_exchange(cx<T> (&v)[kE], int t, T* lr, int lstride)
    {
        constexpr int R = stage_radix(L, kE, s);
        constexpr int Ns = stage_ns(L, kE, s);
        constexpr int NB = kE / R;
        constexpr int R2 = stage_radix(L, kE, s + 1);
        constexpr int NB2 = kE / R2;
        cx<T> w[kE];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            fft_sync<WAVE>();  // previous readers of the scratch are done
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int j = t + q * kT;
                const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    lr[S::lds_slot(base + r * Ns) * lstride] = half ? v[q * R + r].y : v[q * R + r].x;
            }
            fft_sync<WAVE>();
#pragma unroll
            for (int q = 0; q < NB2; ++q) {
                const int j = t + q * kT;
#pragma unroll
                for (int r = 0; r < R2; ++r) {
                    const T x = lr[S::lds_slot(j + r * (L / R2)) * lstride];
                    if (half)
                        w[q * R2 + r].y = x;
                    else
                        w[q * R2 + r].x = x;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kE; ++i) v[i] = w[i];
    }

    template <int s>
    __device__ static __forceinline__ void stage(cx<T> (&v)[kE], int t, cx<T>* lds, int lstride,
                                                 const cx<T>* __restrict__ tw, int twstride)
    {
        constexpr int R = stage_radix(L, kE, s);
        constexpr int Ns = stage_ns(L, kE, s);
        constexpr int NB = kE / R;  // butterflies per thread
        if constexpr (s > 0 && !SPLIT) {
            // read this stage's inputs: element j + r*(L/R) for butterfly j
            fft_sync<WAVE>();
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int j = t + q * kT;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q * R + r] = lds[S::lds_slot(j + r * (L / R)) * lstride];
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int j = t + q * kT;
            if constexpr (Ns > 1) {
                const int jm = j % Ns;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    // exp(DIR 2 pi i r jm / (Ns R)) = w_Lmax^(r jm Lmax/(Ns R)); the
                    // table is small, so a 32-bit byte offset from its base
                    const unsigned ti = (unsigned)((r * jm) * (L / (Ns * R)) * twstride);
                    const cx<T> w = *reinterpret_cast<const cx<T>*>(
                        reinterpret_cast<const char*>(tw) + ti * (unsigned)sizeof(cx<T>));
                    v[q * R + r] = DIR < 0 ? cmul(v[q * R + r], w) : cmulc(v[q * R + r], w);
                }
            }
            dft<R, DIR, HALF_IN && s == 0>(&v[q * R]);
        }
        if constexpr (s + 1 < S::kStages) {
            if constexpr (SPLIT) {
                split_exchange<s>(v, t, reinterpret_cast<T*>(lds), lstride);
            } else {
                fft_sync<WAVE>();  // previous readers of lds are done
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const int j = t + q * kT;
                    const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        lds[S::lds_slot(base + r * Ns) * lstride] = v[q * R + r];
                }
            }
            stage<s + 1>(v, t, lds, lstride, tw, twstride);
        }
    }

    __device__ static __forceinline__ void run(cx<T> (&v)[kE], int t, cx<T>* lds, int lstride,
                                               const cx<T>* __restrict__ tw, int twstride)
    {
        if constexpr (L > 1) stage<0>(v, t, lds, lstride, tw, twstride);
    }
};

}  // namespace mmx
