// Two-level FFT of power-of-two lines held in LDS (N = N1 * N2, both fixed
// at compile time).
//
// With n = N2 a + t and k = k1 + N1 k2 the DFT factorises as
//   X[k1 + N1 k2] = sum_t w_N2^{t k2} ( w_N^{t k1} sum_a x[N2 a + t] w_N1^{a k1} ).
// Phase A: the thread owning column t of a line loads its N1 elements
// (stride N2), takes an N1-point DFT in registers, multiplies by w_N^{t k1}
// and writes them back transposed; phase B: the thread owning row k1 loads
// N2 contiguous values, takes an N2-point DFT in registers and stores
// X[k1 + N1 k2].  Both register DFTs are themselves split the same way
// with constant twiddles, so every index and twiddle position is a
// compile-time constant.  An inverse transform is the same with conjugate
// roots (unnormalised).  Each thread owns at most one column and one row:
// nlines * max(N1, N2) <= blockDim.x.
#pragma once
#include "fft_device.h"

namespace mirve {

// exp(2 pi i m / 32), correctly rounded
__device__ constexpr double kCos32[32] = {1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452, 0.7071067811865476, 0.5555702330196022, 0.3826834323650898, 0.19509032201612828, 0.0, -0.19509032201612828, -0.3826834323650898, -0.5555702330196022, -0.7071067811865476, -0.8314696123025452, -0.9238795325112867, -0.9807852804032304, -1.0, -0.9807852804032304, -0.9238795325112867, -0.8314696123025452, -0.7071067811865476, -0.5555702330196022, -0.3826834323650898, -0.19509032201612828, 0.0, 0.19509032201612828, 0.3826834323650898, 0.5555702330196022, 0.7071067811865476, 0.8314696123025452, 0.9238795325112867, 0.9807852804032304};
__device__ constexpr double kSin32[32] = {0.0, 0.19509032201612828, 0.3826834323650898, 0.5555702330196022, 0.7071067811865476, 0.8314696123025452, 0.9238795325112867, 0.9807852804032304, 1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452, 0.7071067811865476, 0.5555702330196022, 0.3826834323650898, 0.19509032201612828, 0.0, -0.19509032201612828, -0.3826834323650898, -0.5555702330196022, -0.7071067811865476, -0.8314696123025452, -0.9238795325112867, -0.9807852804032304, -1.0, -0.9807852804032304, -0.9238795325112867, -0.8314696123025452, -0.7071067811865476, -0.5555702330196022, -0.3826834323650898, -0.19509032201612828};

template <int L>
__device__ __forceinline__ constexpr int tw_index(int m) { return (m * (32 / L)) & 31; }

// v[j] *= exp(-+2 pi i m / L) with m, L constant
template <typename T, int L>
__device__ __forceinline__ cplx<T> rot_const(cplx<T> a, int m, bool inv) {
    const int idx = tw_index<L>(m);
    const T c = T(kCos32[idx]);
    const T s = inv ? T(kSin32[idx]) : T(-kSin32[idx]);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
}

template <typename T, int L>
struct RegDFT;

template <typename T>
struct RegDFT<T, 2> {
    static __device__ __forceinline__ void run(cplx<T>* v, bool) {
        const cplx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T>
struct RegDFT<T, 4> {
    static __device__ __forceinline__ void run(cplx<T>* v, bool inv) { dft4(v[0], v[1], v[2], v[3], inv); }
};

template <typename T>
struct RegDFT<T, 8> {
    static __device__ __forceinline__ void run(cplx<T>* v, bool inv) {
        cplx<T> (&a)[8] = *reinterpret_cast<cplx<T>(*)[8]>(v);
        dft8(a, inv);
    }
};

// L = A * B with A, B in {2, 4, 8}: same factorisation as the line FFT
template <typename T, int A, int B>
__device__ __forceinline__ void reg_dft_split(cplx<T>* v, bool inv) {
    constexpr int L = A * B;
    cplx<T> y[L];                       // y[b * A + k1]
#pragma unroll
    for (int b = 0; b < B; ++b) {
        cplx<T> u[A];
#pragma unroll
        for (int a = 0; a < A; ++a) u[a] = v[B * a + b];
        RegDFT<T, A>::run(u, inv);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) y[b * A + k1] = (b * k1 == 0) ? u[k1] : rot_const<T, L>(u[k1], b * k1, inv);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cplx<T> u[B];
#pragma unroll
        for (int b = 0; b < B; ++b) u[b] = y[b * A + k1];
        RegDFT<T, B>::run(u, inv);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k2];
    }
}

template <typename T>
struct RegDFT<T, 16> {
    static __device__ __forceinline__ void run(cplx<T>* v, bool inv) { reg_dft_split<T, 4, 4>(v, inv); }
};

template <typename T>
struct RegDFT<T, 32> {
    static __device__ __forceinline__ void run(cplx<T>* v, bool inv) { reg_dft_split<T, 8, 4>(v, inv); }
};

// Split of each supported line length.
template <int N>
struct Split;
template <> struct Split<16> { static constexpr int N1 = 4, N2 = 4; };
template <> struct Split<32> { static constexpr int N1 = 4, N2 = 8; };
template <> struct Split<64> { static constexpr int N1 = 8, N2 = 8; };
template <> struct Split<128> { static constexpr int N1 = 8, N2 = 16; };
template <> struct Split<256> { static constexpr int N1 = 16, N2 = 16; };
template <> struct Split<512> { static constexpr int N1 = 16, N2 = 32; };
template <> struct Split<1024> { static constexpr int N1 = 32, N2 = 32; };

__host__ __device__ constexpr int split_max(int N) {
    return N == 16 ? 4 : N == 32 ? 8 : N == 64 ? 8 : N == 128 ? 16 : N == 256 ? 16 : N == 512 ? 32
         : N == 1024 ? 32 : 0;
}

// In-place DFT of nlines lines (element e of line l at buf[l * LS + lp(e)]),
// natural order in and out.  tw(k1, t) = exp(-2 pi i t k1 / N) is the
// twiddle of column t and output k1 of the first phase: an LDS table
// (LdsTw) or the calling thread's own values in registers (RegTw).
template <typename T, int N, typename TW>
__device__ __forceinline__ void fft_lines_tw(cplx<T>* buf, int nlines, int LS, const TW& tw,
                                             bool inv) {
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    const int tid = threadIdx.x;
    {   // phase A: columns t < N2
        const int line = tid / N2, t = tid % N2;
        const bool act = line < nlines;
        cplx<T> v[N1];
        cplx<T>* L = buf + line * LS;
        if (act) {
#pragma unroll
            for (int a = 0; a < N1; ++a) v[a] = L[lp(N2 * a + t)];
            RegDFT<T, N1>::run(v, inv);
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) {
                cplx<T> w = tw(k1, t);
                if (inv) w.y = -w.y;
                v[k1] = cmul(v[k1], w);
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) L[lp(k1 * N2 + t)] = v[k1];
        }
        __syncthreads();
    }
    {   // phase B: rows k1 < N1
        const int line = tid / N1, k1 = tid % N1;
        const bool act = line < nlines;
        cplx<T> v[N2];
        cplx<T>* L = buf + line * LS;
        if (act) {
#pragma unroll
            for (int b = 0; b < N2; ++b) v[b] = L[lp(k1 * N2 + b)];
            RegDFT<T, N2>::run(v, inv);
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) L[lp(k1 + N1 * k2)] = v[k2];
        }
        __syncthreads();
    }
}

// Phase-A twiddles from an LDS table laid out as N1 x N2,
// tw[k1 * N2 + t], so that the threads of a column group read consecutive
// entries (no bank conflicts).
template <typename T, int N>
struct LdsTw {
    const cplx<T>* tw;
    __device__ __forceinline__ cplx<T> operator()(int k1, int t) const {
        return tw[k1 * Split<N>::N2 + t];
    }
};

// Phase-A twiddles of the calling thread (column t = threadIdx.x mod N2)
// held in registers: w[k1] = exp(-2 pi i t k1 / N).
template <typename T, int N>
struct RegTw {
    const cplx<T> (&w)[Split<N>::N1];
    __device__ __forceinline__ cplx<T> operator()(int k1, int) const { return w[k1]; }
};

// Loads the calling thread's phase-A twiddles from the global table
// tw[m] = exp(-2 pi i m / N).
template <typename T, int N>
__device__ __forceinline__ void load_reg_twiddles(const cplx<T>* tw, cplx<T> (&w)[Split<N>::N1]) {
    const int t = threadIdx.x % Split<N>::N2;
    w[0] = {T(1), T(0)};
#pragma unroll
    for (int k1 = 1; k1 < Split<N>::N1; ++k1) w[k1] = tw[t * k1];
}

template <typename T, int N>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, int nlines, int LS,
                                          const cplx<T>* __restrict__ tw, bool inv) {
    fft_lines_tw<T, N>(buf, nlines, LS, LdsTw<T, N>{tw}, inv);
}

// Line-FFT policies of the kernels: a fixed power-of-two length, or the
// runtime mixed-radix plan with MAXB butterflies per thread.
template <int N_>
struct FastFFT {
    static constexpr bool fast = true;
    static constexpr int N = N_;
    static constexpr int MAXB = 1;
};
template <int MAXB_>
struct GenericFFT {
    static constexpr bool fast = false;
    static constexpr int N = 0;
    static constexpr int MAXB = MAXB_;
};

template <typename T, typename F>
__device__ __forceinline__ void line_fft(cplx<T>* buf, int nlines, int LS, const AxisPlan& pl,
                                         const cplx<T>* __restrict__ tw, bool inv) {
    if constexpr (F::fast) fft_lines<T, F::N>(buf, nlines, LS, tw, inv);
    else lds_fft<T, F::MAXB>(buf, nlines, LS, pl, tw, inv);
}

// Number of phase-A twiddles a thread holds in registers (1 for the runtime
// plans, which read theirs from global memory).
template <typename F, bool = F::fast>
struct RegTwCount {
    static constexpr int n = 1;
};
template <typename F>
struct RegTwCount<F, true> {
    static constexpr int n = Split<F::N>::N1;
};

// Line FFT with the fixed-size plans' twiddles in the calling thread's
// registers (wr, from load_reg_twiddles); the runtime plans use tw.
template <typename T, typename F>
__device__ __forceinline__ void line_fft_rt(cplx<T>* buf, int nlines, int LS, const AxisPlan& pl,
                                            const cplx<T> (&wr)[RegTwCount<F>::n],
                                            const cplx<T>* __restrict__ tw, bool inv) {
    if constexpr (F::fast) fft_lines_tw<T, F::N>(buf, nlines, LS, RegTw<T, F::N>{wr}, inv);
    else lds_fft<T, F::MAXB>(buf, nlines, LS, pl, tw, inv);
}

}  // namespace mirve
