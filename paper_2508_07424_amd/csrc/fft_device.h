// Mixed-radix Stockham FFT over lines held in LDS.
//
// A pass of radix R with span p (the product of the radices already
// applied) maps butterfly i in [0, N/R) of each line as follows: with
// k = i mod p it reads x[i + t N/R] (t < R), multiplies element t by the
// twiddle w_{pR}^{t k}, takes an R-point DFT and writes the results to
// y[(i - k) R + k + t p].  The pass is done in place: every thread first
// gathers its butterflies into registers, the block synchronises, then all
// results are scattered back.  After the last pass the line holds its DFT
// in natural order.  Forward transforms use exp(-2 pi i/N); inverse ones the
// conjugate, unnormalised.
#pragma once
#include "common.h"

namespace mirve {

template <typename T>
__device__ inline cplx<T> mul_mi(cplx<T> a) { return {a.y, -a.x}; }   // a * (-i)
template <typename T>
__device__ inline cplx<T> mul_pi(cplx<T> a) { return {-a.y, a.x}; }   // a * (+i)

template <typename T>
__device__ inline void dft4(cplx<T>& v0, cplx<T>& v1, cplx<T>& v2, cplx<T>& v3, bool inv) {
    cplx<T> a0 = cadd(v0, v2), a1 = csub(v0, v2);
    cplx<T> a2 = cadd(v1, v3), d = csub(v1, v3);
    cplx<T> a3 = inv ? mul_pi(d) : mul_mi(d);
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

template <typename T>
__device__ inline void dft8(cplx<T> (&v)[8], bool inv) {
    const T r = T(0.70710678118654752440084436210485);
    cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, inv);
    dft4(o0, o1, o2, o3, inv);
    cplx<T> t1, t2, t3;
    if (!inv) {
        t1 = {(o1.x + o1.y) * r, (o1.y - o1.x) * r};
        t2 = mul_mi(o2);
        t3 = {(o3.y - o3.x) * r, -(o3.x + o3.y) * r};
    } else {
        t1 = {(o1.x - o1.y) * r, (o1.x + o1.y) * r};
        t2 = mul_pi(o2);
        t3 = {-(o3.x + o3.y) * r, (o3.x - o3.y) * r};
    }
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

// Direct R-point DFT for the odd radices 3, 5, 7.
template <typename T, int R>
__device__ inline void dft_odd(cplx<T> (&v)[8], bool inv) {
    constexpr double PI2 = 6.283185307179586476925286766559;
    cplx<T> out[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        cplx<T> acc = v[0];
#pragma unroll
        for (int t = 1; t < R; ++t) {
            const int m = (t * k) % R;
            const T c = T(__builtin_cos(PI2 * m / R));
            const T s = inv ? T(__builtin_sin(PI2 * m / R)) : T(-__builtin_sin(PI2 * m / R));
            acc.x += v[t].x * c - v[t].y * s;
            acc.y += v[t].x * s + v[t].y * c;
        }
        out[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
}

template <typename T>
__device__ inline void dft_any(cplx<T> (&v)[8], int R, bool inv) {
    switch (R) {
        case 2: {
            cplx<T> a = v[0], b = v[1];
            v[0] = cadd(a, b);
            v[1] = csub(a, b);
            break;
        }
        case 3: dft_odd<T, 3>(v, inv); break;
        case 4: dft4(v[0], v[1], v[2], v[3], inv); break;
        case 5: dft_odd<T, 5>(v, inv); break;
        case 7: dft_odd<T, 7>(v, inv); break;
        case 8: dft8(v, inv); break;
        default: break;
    }
}

// LDS element index of element e of a line: one padding slot after every 16
// elements, so that the strided scatters of the early Stockham passes (stride
// R elements) spread over all banks instead of hitting a few.
__device__ __forceinline__ int lp(int e) { return e + (e >> 4); }

// LDS line stride for lines of N elements (odd, so that walking across lines
// is conflict-free too).
__host__ __device__ inline int lds_line(int N) { return N + (N >> 4) + 1; }

// In-place DFT of `nlines` lines in LDS; element e of line l is at
// buf[l * lstride + lp(e)].  MAXB bounds the butterflies a thread carries
// per pass: nlines * N / min_radix <= MAXB * blockDim.x.
template <typename T, int MAXB>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, int nlines, int lstride, const AxisPlan& pl,
                        const cplx<T>* __restrict__ tw, bool inv) {
    const int N = pl.N;
    int p = 1;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.rad[st];
        const int nb = N / R;
        const int total = nb * nlines;
        const int twstep = N / (p * R);
        cplx<T> v[MAXB][8];
#pragma unroll
        for (int c = 0; c < MAXB; ++c) {
            const int b = threadIdx.x + c * blockDim.x;
            if (b < total) {
                const int line = b / nb, i = b - line * nb;
                const cplx<T>* base = buf + line * lstride;
                const int k = i % p;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (t < R) v[c][t] = base[lp(i + t * nb)];
#pragma unroll
                for (int t = 1; t < 8; ++t) {
                    if (t < R) {
                        cplx<T> w = tw[t * k * twstep];
                        if (inv) w.y = -w.y;
                        v[c][t] = cmul(v[c][t], w);
                    }
                }
                dft_any<T>(v[c], R, inv);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < MAXB; ++c) {
            const int b = threadIdx.x + c * blockDim.x;
            if (b < total) {
                const int line = b / nb, i = b - line * nb;
                cplx<T>* base = buf + line * lstride;
                const int k = i % p;
                const int j = (i - k) * R + k;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (t < R) base[lp(j + t * p)] = v[c][t];
            }
        }
        __syncthreads();
        p *= R;
    }
}

}  // namespace mirve
