// Green-operator pipeline: F^-1{ P(xi) : F[ g(phi) C : eps ] } (Eq. 24 R1,
// Eq. 26) as three kinds of LDS-staged passes over the field.
//
//  x-forward : per block, a few rows along x of all s components.  The
//              prologue evaluates the degraded stress voxel by voxel (Eq. 2,
//              12) -- or the conjugate-gradient direction update fused with
//              it -- and two real rows are packed into one complex line
//              (row 2i in the real part, row 2i+1 in the imaginary part),
//              transformed, and split into their half spectra.
//  axis pass : per block, whole lines of all s components along y (stored
//              contiguously) or a tile of y columns along z (strided by
//              n_y, read in 128-byte rows).  Forward, projection P(n) applied
//              per frequency, inverse, in one visit on the last axis.  y
//              lines of 128, 256 or 512 points can instead go one line
//              position per wave (k_axis_wave), and a Green operator of
//              which only the norm is wanted stops after the projection
//              (k_axis_wave_norm, Parseval).
//  x-inverse : the reverse of the x-forward pass; the epilogue stores the
//              result or applies the conjugate-gradient update in place.
//
// Spectrum layout (per RVE): [c][kx][z][y], kx in [0, n_x/2]: the x passes
// transpose through LDS so that the y lines are contiguous.  A batch of B
// RVEs of the same grid shares every launch (RVE index = last grid index).
#include "kernels.h"
#include "fft2l.h"
#include "reduce.h"

namespace mirve {

// ---------------------------------------------------------------------------
// pointwise helpers
// ---------------------------------------------------------------------------

template <typename T, int S>
__device__ inline void mat_apply(const MatEntry<T>& m, const T (&e)[S], T (&o)[S]) {
#pragma unroll
    for (int a = 0; a < S; ++a) {
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < S; ++b) acc += m.C[a * S + b] * e[b];
        o[a] = acc;
    }
}

template <typename T>
__device__ inline T degr(T phi, T k) {
    const T u = T(1) - phi;
    return u * u + k;
}

// Compatible-strain projection P(n) (Eq. 26, symmetric reading) on one
// Mandel vector of complex spectra.  The direction is passed as the
// frequency x and y = x / |x|^2 (both zero at the zero frequency): with
// n = x / |x| and the symmetric tensor t of the Mandel vector,
// P_ij = n_i u_j + u_i n_j - (n.u) n_i n_j, u = t n, equals
// y_i U_j + U_i y_j - (x.U) y_i y_j with U = t x, which needs no square root.
template <typename T>
__device__ __forceinline__ void project2(cplx<T> (&v)[3], const T (&x)[3], const T (&y)[3]) {
    const T is2 = T(0.70710678118654752440084436210485);
    const T s2 = T(1.4142135623730950488016887242097);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const T a = part ? v[0].y : v[0].x;
        const T b = part ? v[1].y : v[1].x;
        const T c = (part ? v[2].y : v[2].x) * is2;
        const T U1 = a * x[0] + c * x[1], U2 = c * x[0] + b * x[1];
        const T W = x[0] * U1 + x[1] * U2;
        const T p0 = T(2) * y[0] * U1 - W * y[0] * y[0];
        const T p1 = T(2) * y[1] * U2 - W * y[1] * y[1];
        const T p2 = s2 * (y[0] * U2 + y[1] * U1 - W * y[0] * y[1]);
        if (part) { v[0].y = p0; v[1].y = p1; v[2].y = p2; }
        else { v[0].x = p0; v[1].x = p1; v[2].x = p2; }
    }
}

template <typename T>
__device__ __forceinline__ void project3(cplx<T> (&v)[6], const T (&x)[3], const T (&y)[3]) {
    const T is2 = T(0.70710678118654752440084436210485);
    const T s2 = T(1.4142135623730950488016887242097);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        T q[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) q[a] = part ? v[a].y : v[a].x;
        const T t[3][3] = {{q[0], q[5] * is2, q[4] * is2},
                           {q[5] * is2, q[1], q[3] * is2},
                           {q[4] * is2, q[3] * is2, q[2]}};
        T U[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) U[i] = t[i][0] * x[0] + t[i][1] * x[1] + t[i][2] * x[2];
        const T W = x[0] * U[0] + x[1] * U[1] + x[2] * U[2];
        auto P = [&](int i, int j) { return y[i] * U[j] + U[i] * y[j] - W * y[i] * y[j]; };
        const T o[6] = {P(0, 0), P(1, 1), P(2, 2), s2 * P(1, 2), s2 * P(0, 2), s2 * P(0, 1)};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            if (part) v[a].y = o[a];
            else v[a].x = o[a];
        }
    }
}

__device__ __forceinline__ int signed_k(int k, int N) { return (2 * k < N) ? k : k - N; }

// Frequency with the Nyquist rule: on an even axis the index k = -N/2
// keeps its frequency only if every other index is zero.  Same h on every
// axis, so x_j = k_j / N_j up to a common factor (rN_j = 1 / N_j); returns
// x and y = x / |x|^2, both zero at the zero frequency.
template <typename T>
__device__ __forceinline__ void freq_xy(const Geom& g, int kx, int ky, int kz, const T (&rN)[3],
                                        T (&x)[3], T (&y)[3]) {
    int sx = (g.nx % 2 == 0 && 2 * kx == g.nx) ? -g.nx / 2 : kx;
    int sy = signed_k(ky, g.ny);
    int sz = g.dim == 3 ? signed_k(kz, g.nz) : 0;
    // the tests use the original indices (a corner with several Nyquist
    // indices loses all of them)
    const int ox = sx, oy = sy, oz = sz;
    const bool nyx = (g.nx % 2 == 0) && (ox == -g.nx / 2);
    const bool nyy = (g.ny % 2 == 0) && (oy == -g.ny / 2);
    const bool nyz = g.dim == 3 && (g.nz % 2 == 0) && (oz == -g.nz / 2);
    if (nyx && (oy != 0 || oz != 0)) sx = 0;
    if (nyy && (ox != 0 || oz != 0)) sy = 0;
    if (nyz && (ox != 0 || oy != 0)) sz = 0;
    x[0] = T(sx) * rN[0];
    x[1] = T(sy) * rN[1];
    x[2] = T(sz) * rN[2];
    const T n2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const T inv = n2 > T(0) ? T(1) / n2 : T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = x[i] * inv;
}

// Symbol of the damage preconditioner at frequency (kx, ky, kz):
// 1 / (abar + bbar |d|^2), |d|^2 the sum over the axes of the tabulated
// |d_j(k_j)|^2 = 4 sin^2(pi k_j / N_j) / h^2 of the forward differences of the
// damage operator (Sec. 4.1, Eq. 24 R2).
template <typename T>
__device__ __forceinline__ T precond_symbol(const Geom& g, const T* dsq, int kx, int ky, int kz,
                                            double abar, double bbar) {
    const T d2 = dsq[kx] + dsq[g.nx + ky] + (g.dim == 3 ? dsq[g.nx + g.ny + kz] : T(0));
    return T(1) / (T(abar) + T(bbar) * d2);
}

// Line length of a pass: a compile-time constant for the fixed-size FFTs, so
// that index arithmetic on it folds into shifts; the runtime plan otherwise.
template <typename F>
__device__ __forceinline__ int line_len(const AxisPlan& pl) {
    if constexpr (F::fast) return F::N;
    else return pl.N;
}

// Global loads each thread keeps in flight in the gather loops of the passes.
constexpr int kLd = 4;

// Loads and stores of the voxel vectors that a pass streams once: with NT,
// non-temporal (the lines are not kept in the caches, which leaves the
// last-level cache to the transposed spectrum that the next pass reads).
template <bool NT, typename T>
__device__ __forceinline__ T ld_s(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_s(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Two adjacent complex values (the same frequency of rows 2i and 2i+1 of the
// transposed spectrum) at a 16-byte-aligned address: one access in FP32.
template <typename T>
__device__ __forceinline__ void ld_pair(const cplx<T>* p, cplx<T>& a, cplx<T>& b) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        a = {T(v.x), T(v.y)};
        b = {T(v.z), T(v.w)};
    } else {
        a = p[0];
        b = p[1];
    }
}
template <typename T>
__device__ __forceinline__ void st_pair(cplx<T>* p, cplx<T> a, cplx<T> b) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(float(a.x), float(a.y), float(b.x), float(b.y));
    } else {
        p[0] = a;
        p[1] = b;
    }
}

// Twiddles of the fixed-size FFTs, loaded once per block (global twiddle
// loads inside the butterflies would each wait on memory).  Each thread
// needs exp(-2 pi i t k1 / N) for its first-phase column t and k1 < N1.
// The x passes, and the axis passes in FP64, whose blocks are limited by
// LDS, keep these in registers (load_reg_twiddles).  The axis passes in
// FP32, limited by registers, keep an LDS table at the start of the dynamic
// LDS whose entry k1 * N2 + t holds that value (stage_twiddles; the host
// sizes every pass's LDS to match).  The runtime plans read theirs from
// global memory.
template <typename F>
__device__ __forceinline__ constexpr int tw_lds_len() { return F::fast ? F::N : 0; }

// Axis passes: registers in FP64, the LDS table in FP32.
template <typename T, typename F>
__device__ __forceinline__ constexpr bool reg_twiddles() {
    return F::fast && sizeof(T) == 8;
}

// x passes: registers in both precisions.
template <typename F>
__device__ __forceinline__ constexpr bool x_reg_twiddles() {
    return F::fast;
}

template <typename T, typename F>
__device__ __forceinline__ void stage_twiddles(cplx<T>* twl, const cplx<T>* tw) {
    if constexpr (F::fast) {
        constexpr int N2 = Split<F::N>::N2;
        for (int i0 = threadIdx.x; i0 < F::N; i0 += kLd * blockDim.x) {
            cplx<T> t[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int i = i0 + u * blockDim.x;
                const int k1 = i / N2, c = i - k1 * N2;
                t[u] = tw[i < F::N ? c * k1 : 0];
            }
            loads_issued();
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int i = i0 + u * blockDim.x;
                if (i < F::N) twl[i] = t[u];
            }
        }
    }
}

// Consecutive workgroups of a launch go to the eight XCDs in turn, and each
// XCD has its own L2.  Renumbering the x index so that the workgroups one XCD
// receives cover consecutive row groups lets neighbouring groups, which share
// the cache lines of the transposed spectrum, meet in the same L2.  A
// bijection of [0, n) when n is a multiple of 8, else the identity.
__device__ __forceinline__ int xcd_group(int bx, int n) {
    if (n & 7) return bx;
    return (bx & 7) * (n >> 3) + (bx >> 3);
}

// ---------------------------------------------------------------------------
// x-forward pass
// ---------------------------------------------------------------------------

template <typename T, int S, int MODE, typename F, bool NT>
__global__ void __launch_bounds__(256) k_xfwd(XfwdArgs<T> a) {
    constexpr bool RT = x_reg_twiddles<F>();
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* const twl = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* buf = twl + (RT ? 0 : tw_lds_len<F>());
    const cplx<T>* const twp = (F::fast && !RT) ? twl : a.tw;
    const Geom& g = a.g;
    const int b = blockIdx.y;
    const int k = a.iter;
    constexpr bool PCG = MODE == XF_PCG || MODE == XF_PCG0;
    constexpr bool CGM = MODE == XF_CG || MODE == XF_CG_T;
    if (CGM) {
        // a solve that stopped in an earlier launch; conv == k (k > 0) is
        // this launch's own stop, whose blocks still apply the last x update
        const int cv = a.cg[b].conv;
        if (k == 0 ? cv <= 0 : cv < k) return;
    } else if (PCG) {
        if (a.pcg[b].conv <= k) return;
    } else if (a.active && !a.active[b]) {
        return;
    }
    const int nx = line_len<F>(a.pl), ny = g.ny, nz = g.nz;
    const int nrows = ny * nz;
    const int RB = a.rows_per_block;          // a power of two
    const int npairs = RB / 2;
    const int lgp = __builtin_ctz(npairs);
    const int grp = xcd_group(blockIdx.x, gridDim.x);
    const int r0 = grp * RB;
    const int LS = lds_line(nx);
    const long long N = g.N;
    const long long so = (long long)b * N;
    const long long fo = so * S;
    const MatEntry<T>* mat = a.mat + (long long)b * g.mstride;
    const uint16_t* mid = a.mat_id + so;
    const T* phi = a.phi + so;

    // CG: the update x += alpha_{k-1} p_{k-1} of the previous iteration
    // (alpha from the p.Ap partials of the previous x-forward pass, the same
    // bits the x-inverse pass used for r), then beta = rr_k / rr_{k-1} and the
    // stopping test from the r.r partials of the previous x-inverse pass.
    // PCG: alpha = rz_k / p.q.
    T beta = T(0), alpha = T(0), alpha_x = T(0);
    bool first = false, stop_now = false;
    if (CGM) {
        const CgDev& cg = a.cg[b];
        if (cg.max_it < 0) {
            beta = T(0.5);                       // timing run: alpha_x = 0
        } else if (k == 0) {
            first = true;
        } else {
            double rr[1], pap[1];
            block_sum_all<1>(a.rr_part + (long long)b * a.nblocks, 0, a.nblocks, rr);
            block_sum_all<1>(a.pap_prev + (long long)b * a.nblocks, 0, a.nblocks, pap);
            const double prev = cg.rr_hist[(k - 1) & 1];
            alpha_x = T(prev / pap[0]);
            int stop = 0;
            if (!isfinite(rr[0])) stop = 2;
            else if (rr[0] <= cg.tol2 * cg.bn2) stop = 1;
            else if (k >= cg.max_it) stop = 3;
            if (threadIdx.x == 0) {
                CgDev* w = const_cast<CgDev*>(a.cg) + b;
                w->rr_hist[k & 1] = rr[0];
                w->rr = rr[0];
                if (stop) {
                    w->status = stop;
                    w->conv = k;
                }
            }
            stop_now = stop != 0;
            beta = T(rr[0] / prev);
        }
    } else if (MODE == XF_PCG) {
        double pq[1];
        block_sum_all<1>(a.pq_part + (long long)b * a.pq_stride, 0, a.pq_n, pq);
        if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
            if (threadIdx.x == 0) {
                a.pcg[b].status = 2;
                a.pcg[b].conv = k;
            }
            return;
        }
        alpha = T(a.pcg[b].rz_hist[k & 1] / pq[0]);
    }
    if constexpr (CGM) {
        if (stop_now) {      // the solve ends here: only the last x update
            for (int v = threadIdx.x; v < RB * nx; v += blockDim.x) {
                const int row = r0 + v / nx;
                if (row >= nrows) continue;
                const long long idx = (long long)row * nx + (v - (v / nx) * nx);
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const long long o = fo + c * N + idx;
                    a.x[o] += alpha_x * a.p[o];
                }
            }
            return;
        }
    }
    // U voxels per thread and round, in three phases: (1) every global load
    // of the round, unconditional at clamped addresses so that none waits
    // for another; (2) the Krylov updates and their stores; (3) the
    // constitutive law, whose material-table loads then meet no global store
    // (a store may alias a load as far as the compiler knows) and can all be
    // issued together, and the LDS tile.
    constexpr int U = S == 6 ? 2 : 4;
    const int tot = RB * nx;
    cplx<T> wr[RegTwCount<F>::n];
    if constexpr (RT) load_reg_twiddles<T, F::N>(a.tw, wr);
    else stage_twiddles<T, F>(twl, a.tw);     // ordered by the barrier before the FFT
    double part = 0.0;
    for (int v0 = threadIdx.x; v0 < tot; v0 += U * blockDim.x) {
        T in0[U][S], in1[U][S], in2[U][S], in3[U], in4[U], ph[U];
        int mv[U];
        long long ix[U];
        bool ok[U];
        // ---- (1) loads
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * blockDim.x;
            const int rl = v / nx, x = v - rl * nx;
            const int row = r0 + rl;
            ok[u] = v < tot && row < nrows;
            const long long idx = (long long)(ok[u] ? row : 0) * nx + x;
            ix[u] = idx;
            if constexpr (PCG) {
                const long long o = so + idx;
                in0[u][0] = ld_s<NT>(a.r + o);
                in4[u] = a.sc[o];
                if constexpr (MODE == XF_PCG) {
                    in1[u][0] = ld_s<NT>(a.x + o);
                    in2[u][0] = ld_s<NT>(a.pd + o);
                    in3[u] = ld_s<NT>(a.q + o);
                }
            } else {
                mv[u] = mid[idx];
                ph[u] = ld_s<NT>(phi + idx);
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const long long o = fo + c * N + idx;
                    if constexpr (CGM) {
                        in0[u][c] = ld_s<NT>(a.r + o);
                        if (!first) {
                            in1[u][c] = ld_s<NT>(a.p + o);
                            in2[u][c] = ld_s<NT>(a.x + o);
                        }
                    } else {
                        in0[u][c] = a.eps ? a.eps[o] : T(0);
                    }
                }
                if constexpr (MODE == XF_CG_T) in3[u] = T(a.tmask[so + idx]);
            }
        }
        loads_issued();
        // ---- (2) Krylov updates; in0 becomes the strain the law acts on
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const long long idx = ix[u];
            if constexpr (PCG) {
                // damage PCG: x += alpha p, r -= alpha q; transform sc * r
                if constexpr (MODE == XF_PCG) {
                    const long long o = so + idx;
                    st_s<NT>(a.x + o, in1[u][0] + alpha * in2[u][0]);
                    in0[u][0] -= alpha * in3[u];
                    st_s<NT>(a.r + o, in0[u][0]);
                }
            } else if constexpr (CGM) {
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const long long o = fo + c * N + idx;
                    if (!first) {
                        st_s<NT>(a.x + o, in2[u][c] + alpha_x * in1[u][c]);
                        in0[u][c] = in0[u][c] + beta * in1[u][c];
                    }
                    st_s<NT>(a.p + o, in0[u][c]);
                }
            } else {
#pragma unroll
                for (int c = 0; c < S; ++c) in0[u][c] = in0[u][c] + a.fcoef * a.f[c];
                if constexpr (MODE == XF_SPLIT) {
                    constexpr int NI = S == 3 ? 2 : 3;
                    T tr = T(0);
#pragma unroll
                    for (int c = 0; c < NI; ++c) tr += in0[u][c];
                    in3[u] = tr > T(0) ? T(1) : T(0);
                    a.tmask[so + idx] = tr > T(0) ? 1 : 0;
                }
            }
        }
        // ---- (3) constitutive law and the LDS tile
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * blockDim.x;
            if (v >= tot) break;
            const int rl = v / nx, x = v - rl * nx;
            T sig[S];
            if (ok[u] && PCG) {
                part += double(in0[u][0]) * double(in0[u][0]);
                sig[0] = in4[u] * in0[u][0];
            } else if (ok[u]) {
                const MatEntry<T>& m = mat[mv[u]];
                const T gg = degr(ph[u], T(g.k_res));
                const T (&e)[S] = in0[u];
                T o[S];
                mat_apply<T, S>(m, e, o);
#pragma unroll
                for (int c = 0; c < S; ++c) sig[c] = gg * o[c];
                if constexpr (MODE == XF_SPLIT || MODE == XF_CG_T) {
                    // sigma = g (C:e - K tr e I) + w K tr e I with w = g where
                    // the (Newton-point) trace is tensile, 1 where it is not:
                    // the split law itself for XF_SPLIT, its tangent for XF_CG_T
                    constexpr int NI = S == 3 ? 2 : 3;
                    T tr = T(0);
#pragma unroll
                    for (int c = 0; c < NI; ++c) tr += e[c];
                    const bool ten = in3[u] != T(0);
                    const T add = ((ten ? gg : T(1)) - gg) * m.K * tr;
#pragma unroll
                    for (int c = 0; c < NI; ++c) sig[c] += add;
                }
                if constexpr (CGM) {
#pragma unroll
                    for (int c = 0; c < S; ++c) part += double(e[c]) * double(sig[c]);
                }
            } else {
#pragma unroll
                for (int c = 0; c < S; ++c) sig[c] = T(0);
            }
#pragma unroll
            for (int c = 0; c < S; ++c) {
                cplx<T>& dst = buf[(c * npairs + (rl >> 1)) * LS + lp(x)];
                if (rl & 1) dst.y = sig[c];
                else dst.x = sig[c];
            }
        }
    }
    __syncthreads();
    if constexpr (RT) line_fft_rt<T, F>(buf, S * npairs, LS, a.pl, wr, twp, false);
    else line_fft<T, F>(buf, S * npairs, LS, a.pl, twp, false);

    // split the packed lines into the half spectra of their two rows and
    // store them transposed: consecutive threads write consecutive y
    const int nxh = nx / 2 + 1;
    cplx<T>* sp = a.spec + (long long)b * S * g.Nspec;
    for (int e = threadIdx.x; e < S * npairs * nxh; e += blockDim.x) {
        const int pr = e & (npairs - 1);
        const int q = e >> lgp;               // q = c * nxh + k
        const int c = q / nxh;
        const int k = q - c * nxh;
        const int line = c * npairs + pr;
        const cplx<T> z = buf[line * LS + lp(k)];
        const cplx<T> zm = buf[line * LS + lp(k == 0 ? 0 : nx - k)];
        // A = (Z_k + conj Z_{-k}) / 2 ;  B = (Z_k - conj Z_{-k}) / (2i)
        const cplx<T> A = {T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
        const cplx<T> Bv = {T(0.5) * (z.y + zm.y), T(-0.5) * (z.x - zm.x)};
        const int rowA = r0 + 2 * pr;
        cplx<T>* spc = sp + (long long)c * g.Nspec + (long long)k * nz * ny;
        if (sizeof(T) == 4 && (nrows & 1) == 0) {   // rows 2i, 2i+1 adjacent and 16-byte aligned
            if (rowA < nrows) st_pair(spc + rowA, A, Bv);
        } else {
            if (rowA < nrows) spc[rowA] = A;        // rowA = z * ny + y
            if (rowA + 1 < nrows) spc[rowA + 1] = Bv;
        }
    }
    if (MODE != XF_GREEN && MODE != XF_SPLIT) {
        double pv[1] = {part};
        block_sum_store<1>(pv, a.partials + (long long)b * a.nblocks, 0, grp);
    }
}

// ---------------------------------------------------------------------------
// axis pass: forward, [projection], inverse along y (contiguous lines) or z
// ---------------------------------------------------------------------------

// (NT is unused: the axis passes touch only the spectrum.)  The fixed-size
// FFTs take their phase-A twiddles from registers in FP64, where LDS limits
// the blocks per CU, and from the LDS table in FP32, where registers do.
template <typename T, int S, int MODE, typename F, bool NT>
__global__ void __launch_bounds__(256) k_axis(AxisArgs<T> a) {
    constexpr bool RT = reg_twiddles<T, F>();
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* const twl = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* buf = twl + (RT ? 0 : tw_lds_len<F>());
    const cplx<T>* const twp = (F::fast && !RT) ? twl : a.tw;
    const Geom& g = a.g;
    const int b = blockIdx.z;
    if (a.cg && a.cg[b].conv <= a.iter) return;
    if (a.pcg && a.pcg[b].conv <= a.iter) return;
    if (a.active && !a.active[b]) return;
    const int TL = a.lines;                   // a power of two
    const int lgt = __builtin_ctz(TL);
    const int Na = line_len<F>(a.pl);
    const int ny = g.ny, nz = g.nz;
    cplx<T>* sp = a.spec + (long long)b * S * g.Nspec;
    const bool inv_only = MODE == AX_INV;
    const T rN[3] = {T(1) / T(g.nx), T(1) / T(g.ny), T(1) / T(g.nz)};
    cplx<T> wr[RegTwCount<F>::n];
    if constexpr (RT) load_reg_twiddles<T, F::N>(a.tw, wr);
    else stage_twiddles<T, F>(twl, a.tw);     // ordered by the barrier before the FFT

    const int LS = lds_line(Na);
    auto fft = [&](int nl, bool inv) {
        if constexpr (RT) line_fft_rt<T, F>(buf, nl, LS, a.pl, wr, twp, inv);
        else line_fft<T, F>(buf, nl, LS, a.pl, twp, inv);
    };
    if (a.contiguous) {
        // lines L = kx * nz + z, element y; LDS line (c, tl)
        const long long nlines = (long long)g.nxh * nz;
        const long long L0 = (long long)blockIdx.x * TL;
        const int tot = S * TL * Na;
        // kLd loads per thread in flight before their LDS writes
        for (int e0 = threadIdx.x; e0 < tot; e0 += kLd * blockDim.x) {
            cplx<T> t[kLd];
            bool in[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {     // unconditional loads at clamped addresses
                const int e = e0 + u * blockDim.x;
                const int q = e / Na, j = e - q * Na, tl = q & (TL - 1), c = q >> lgt;
                const long long L = L0 + tl;
                in[u] = e < tot && L < nlines;
                t[u] = sp[in[u] ? (long long)c * g.Nspec + L * ny + j : 0];
            }
            loads_issued();
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int e = e0 + u * blockDim.x;
                const int q = e / Na, j = e - q * Na, tl = q & (TL - 1), c = q >> lgt;
                if (e < tot)
                    buf[(c * TL + tl) * LS + lp(j)] = {in[u] ? t[u].x : T(0), in[u] ? t[u].y : T(0)};
            }
        }
        __syncthreads();
        fft(S * TL, inv_only);
        if constexpr (MODE == AX_FWD_M_INV) {
            const double abar = a.pcg[b].abar, bbar = a.pcg[b].bbar;
            for (int e = threadIdx.x; e < S * TL * Na; e += blockDim.x) {
                const int q = e / Na, j = e - q * Na, tl = q & (TL - 1), c = q >> lgt;
                const long long L = L0 + tl;
                if (L >= nlines) continue;
                const T m = precond_symbol<T>(g, a.dsq, (int)(L / nz), j, (int)(L % nz), abar, bbar);
                cplx<T>& v = buf[(c * TL + tl) * LS + lp(j)];
                v.x *= m;
                v.y *= m;
            }
            __syncthreads();
            fft(S * TL, true);
        }
        if constexpr (MODE == AX_FWD_P_INV) {
            for (int e = threadIdx.x; e < TL * Na; e += blockDim.x) {
                const int tl = e / Na, j = e - tl * Na;
                const long long L = L0 + tl;
                if (L >= nlines) continue;
                const int kx = (int)(L / nz), kz = (int)(L % nz);
                T fx[3], fy[3];
                freq_xy<T>(g, kx, j, kz, rN, fx, fy);
                cplx<T> v[S];
#pragma unroll
                for (int c = 0; c < S; ++c) v[c] = buf[(c * TL + tl) * LS + lp(j)];
                if constexpr (S == 3) project2<T>(v, fx, fy);
                else if constexpr (S == 6) project3<T>(v, fx, fy);
#pragma unroll
                for (int c = 0; c < S; ++c) buf[(c * TL + tl) * LS + lp(j)] = v[c];
            }
            __syncthreads();
            fft(S * TL, true);
        }
        for (int e = threadIdx.x; e < S * TL * Na; e += blockDim.x) {
            const int q = e / Na, j = e - q * Na, tl = q & (TL - 1), c = q >> lgt;
            const long long L = L0 + tl;
            if (L < nlines) sp[(long long)c * g.Nspec + L * ny + j] = buf[(c * TL + tl) * LS + lp(j)];
        }
    } else {
        // z lines at fixed (kx, y), y in a tile of TL columns; LDS line (c, tl)
        const int nyt = (ny + TL - 1) / TL;
        const int tile = xcd_group(blockIdx.x, gridDim.x);
        const int kx = tile / nyt;
        const int y0 = (tile % nyt) * TL;
        const int W = S * TL;
        const long long base = (long long)kx * nz * ny + y0;
        const int tot = W * Na;
        for (int e0 = threadIdx.x; e0 < tot; e0 += kLd * blockDim.x) {
            cplx<T> t[kLd];
            bool in[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {     // unconditional loads at clamped addresses
                const int e = e0 + u * blockDim.x;
                const int tl = e & (TL - 1), q = e >> lgt, j = q / S, c = q - j * S;
                in[u] = e < tot && y0 + tl < ny;
                t[u] = sp[in[u] ? (long long)c * g.Nspec + base + (long long)j * ny + tl : 0];
            }
            loads_issued();
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int e = e0 + u * blockDim.x;
                const int tl = e & (TL - 1), q = e >> lgt, j = q / S, c = q - j * S;
                if (e < tot)
                    buf[(c * TL + tl) * LS + lp(j)] = {in[u] ? t[u].x : T(0), in[u] ? t[u].y : T(0)};
            }
        }
        __syncthreads();
        fft(W, inv_only);
        if constexpr (MODE == AX_FWD_M_INV) {
            const double abar = a.pcg[b].abar, bbar = a.pcg[b].bbar;
            for (int e = threadIdx.x; e < W * Na; e += blockDim.x) {
                const int tl = e & (TL - 1), q = e >> lgt, j = q / S, c = q - j * S;
                if (y0 + tl >= ny) continue;
                const T m = precond_symbol<T>(g, a.dsq, kx, y0 + tl, j, abar, bbar);
                cplx<T>& v = buf[(c * TL + tl) * LS + lp(j)];
                v.x *= m;
                v.y *= m;
            }
            __syncthreads();
            fft(W, true);
        }
        if constexpr (MODE == AX_FWD_P_INV) {
            for (int e = threadIdx.x; e < TL * Na; e += blockDim.x) {
                const int tl = e & (TL - 1), j = e >> lgt;
                if (y0 + tl >= ny) continue;
                T fx[3], fy[3];
                freq_xy<T>(g, kx, y0 + tl, j, rN, fx, fy);
                cplx<T> v[S];
#pragma unroll
                for (int c = 0; c < S; ++c) v[c] = buf[(c * TL + tl) * LS + lp(j)];
                if constexpr (S == 3) project2<T>(v, fx, fy);
                else if constexpr (S == 6) project3<T>(v, fx, fy);
#pragma unroll
                for (int c = 0; c < S; ++c) buf[(c * TL + tl) * LS + lp(j)] = v[c];
            }
            __syncthreads();
            fft(W, true);
        }
        for (int e = threadIdx.x; e < W * Na; e += blockDim.x) {
            const int tl = e & (TL - 1), q = e >> lgt, j = q / S, c = q - j * S;
            if (y0 + tl < ny)
                sp[(long long)c * g.Nspec + base + (long long)j * ny + tl] = buf[(c * TL + tl) * LS + lp(j)];
        }
    }
}

// ---------------------------------------------------------------------------
// one-wave axis pass: whole y lines in the registers of one wave
// ---------------------------------------------------------------------------
//
// For contiguous lines of N = 128, 256 or 512 points, LN lanes of a wave
// (64, or 32 for N = 128, so that a wave carries two lines) own one line
// position for all S components, and no LDS or barrier is shared with the
// other waves of the block.  Lane l of a line holds x[l + LN m], m < V
// (V = N / LN values).  Each line is a Stockham FFT of P passes (512 = 8^3,
// 256 = 4^4, 128 = 4^3 2) with V / R butterflies of radix R per lane: in the
// pass of span p, butterfly i reads x[i + t N/R], t < R, multiplies element
// t by w_{pR}^{t k} (k = i mod p), takes an R-point DFT and writes
// y[(i - k) R + k + t p].  Butterfly i = l + LN j reads exactly the lane's
// values m = j + t V/R, so the first pass reads the line straight from HBM
// (coalesced runs); between passes the line goes through the wave's own LDS
// region; after the last pass (p = N/R) the lane again holds X[l + LN m].
// So the lane holds the same frequencies of every component, and the
// projection (or the damage preconditioner) is applied in registers.  The
// inverse runs the same passes with conjugate twiddles from that layout and
// ends in it, so every load and store is a coalesced run.

// Orders the LDS accesses of the lanes of one wave (no block barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
struct WavePlan {
    static constexpr int LN = N >= 256 ? 64 : 32;          // lanes per line
    static constexpr int V = N / LN;                      // values per lane
    static constexpr int P = N == 512 ? 3 : 4;            // passes
    static constexpr int radix(int s) { return (N == 128 && s == 3) ? 2 : V; }
    static constexpr int span(int s) {
        int p = 1;
        for (int u = 0; u < s; ++u) p *= radix(u);
        return p;
    }
    // offset of pass s's twiddles (passes 1 .. P-1) in the lane's table
    static constexpr int tw_off(int s) {
        int o = 0;
        for (int u = 1; u < s; ++u) o += (V / radix(u)) * (radix(u) - 1);
        return o;
    }
    static constexpr int NTW = tw_off(P);
};

template <typename T, int R>
__device__ __forceinline__ void wave_dft(cplx<T> (&u)[R], bool inv) {
    if constexpr (R == 8) dft8(u, inv);
    else if constexpr (R == 4) dft4(u[0], u[1], u[2], u[3], inv);
    else {
        const cplx<T> a = u[0], b = u[1];
        u[0] = cadd(a, b);
        u[1] = csub(a, b);
    }
}

// Pass s of the line FFT of the calling lane (l = lane within its line).
template <typename T, int N, int s>
__device__ __forceinline__ void wave_pass(cplx<T> (&v)[WavePlan<N>::V],
                                          const cplx<T> (&wtw)[WavePlan<N>::NTW], cplx<T>* lds,
                                          int l, bool inv) {
    using WP = WavePlan<N>;
    constexpr int R = WP::radix(s), p = WP::span(s), NB = WP::V / R;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        cplx<T> u[R];
#pragma unroll
        for (int t = 0; t < R; ++t) u[t] = v[j + t * NB];
        if constexpr (s > 0) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                const cplx<T> w = wtw[WP::tw_off(s) + j * (R - 1) + t - 1], x = u[t];
                u[t] = inv ? cplx<T>{x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y}   // x conj(w)
                           : cplx<T>{x.x * w.x - x.y * w.y, x.y * w.x + x.x * w.y};
            }
        }
        wave_dft<T, R>(u, inv);
#pragma unroll
        for (int t = 0; t < R; ++t) v[j + t * NB] = u[t];
    }
    if constexpr (s < WP::P - 1) {
        wave_lds_sync();                          // earlier reads of the region are done
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = l + WP::LN * j, k = i & (p - 1);
            const int base = (i - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) lds[lp(base + t * p)] = v[j + t * NB];
        }
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < WP::V; ++m) v[m] = lds[lp(l + WP::LN * m)];
    }
}

template <typename T, int N>
__device__ __forceinline__ void wave_line_fft(cplx<T> (&v)[WavePlan<N>::V],
                                              const cplx<T> (&wtw)[WavePlan<N>::NTW], cplx<T>* lds,
                                              int l, bool inv) {
    wave_pass<T, N, 0>(v, wtw, lds, l, inv);
    wave_pass<T, N, 1>(v, wtw, lds, l, inv);
    wave_pass<T, N, 2>(v, wtw, lds, l, inv);
    if constexpr (WavePlan<N>::P > 3) wave_pass<T, N, 3>(v, wtw, lds, l, inv);
}

// Twiddles of passes 1 .. P-1 of the calling lane (l = lane within its
// line): w_{pR}^{t k} = tw[t k N / (p R)], tw[m] = exp(-2 pi i m / N).
template <typename T, int N>
__device__ __forceinline__ void wave_twiddles(const cplx<T>* __restrict__ tw, int l,
                                              cplx<T> (&wtw)[WavePlan<N>::NTW]) {
    using WP = WavePlan<N>;
#pragma unroll
    for (int s = 1; s < WP::P; ++s) {
        const int R = WP::radix(s), p = WP::span(s), NB = WP::V / R, stride = N / (p * R);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = (l + WP::LN * j) & (p - 1);
#pragma unroll
            for (int t = 1; t < R; ++t) wtw[WP::tw_off(s) + j * (R - 1) + t - 1] = tw[t * k * stride];
        }
    }
}

// MODE: AX_FWD or AX_INV (one direction, any S), AX_FWD_P_INV (S = 3,
// projection) or AX_FWD_M_INV (S = 1, damage preconditioner).  Four waves
// per block.
template <typename T, int S, int MODE, int N>
__global__ void __launch_bounds__(256) k_axis_wave(AxisArgs<T> a) {
    using WP = WavePlan<N>;
    constexpr int V = WP::V, LN = WP::LN, LPW = 64 / LN;
    extern __shared__ unsigned char smem_raw[];
    const Geom& g = a.g;
    const int b = blockIdx.z;
    if (a.cg && a.cg[b].conv <= a.iter) return;
    if (a.pcg && a.pcg[b].conv <= a.iter) return;
    if (a.active && !a.active[b]) return;
    const int lane = threadIdx.x & 63, l = lane & (LN - 1), gl = lane / LN;
    const int wv = threadIdx.x >> 6;
    const long long L = ((long long)blockIdx.x * (blockDim.x >> 6) + wv) * LPW + gl;   // kx * nz + z
    const long long nlines = (long long)g.nxh * g.nz;
    if (L >= nlines) return;                      // no barrier follows
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw) + (wv * LPW + gl) * lds_line(N);
    cplx<T>* sp = a.spec + (long long)b * S * g.Nspec + L * N;   // n_y == N

    cplx<T> v[S][V];
#pragma unroll
    for (int c = 0; c < S; ++c)
#pragma unroll
        for (int m = 0; m < V; ++m) v[c][m] = sp[(long long)c * g.Nspec + l + LN * m];

    cplx<T> wtw[WP::NTW];
    wave_twiddles<T, N>(a.tw, l, wtw);

    constexpr bool FWD = MODE != AX_INV;
    if constexpr (FWD) {
#pragma unroll
        for (int c = 0; c < S; ++c) wave_line_fft<T, N>(v[c], wtw, lds, l, false);
    }
    const int kx = (int)(L / g.nz), kz = (int)(L - (long long)kx * g.nz);
    if constexpr (MODE == AX_FWD_P_INV) {
        const T rN[3] = {T(1) / T(g.nx), T(1) / T(g.ny), T(1) / T(g.nz)};
#pragma unroll
        for (int m = 0; m < V; ++m) {
            T fx[3], fy[3];
            freq_xy<T>(g, kx, l + LN * m, kz, rN, fx, fy);
            cplx<T> u[S];
#pragma unroll
            for (int c = 0; c < S; ++c) u[c] = v[c][m];
            if constexpr (S == 3) project2<T>(u, fx, fy);
            else project3<T>(u, fx, fy);
#pragma unroll
            for (int c = 0; c < S; ++c) v[c][m] = u[c];
        }
    } else if constexpr (MODE == AX_FWD_M_INV) {
        const double abar = a.pcg[b].abar, bbar = a.pcg[b].bbar;
#pragma unroll
        for (int m = 0; m < V; ++m) {
            const T mul = precond_symbol<T>(g, a.dsq, kx, l + LN * m, kz, abar, bbar);
            v[0][m].x *= mul;
            v[0][m].y *= mul;
        }
    }
    if constexpr (MODE != AX_FWD) {
#pragma unroll
        for (int c = 0; c < S; ++c) wave_line_fft<T, N>(v[c], wtw, lds, l, true);
    }
#pragma unroll
    for (int c = 0; c < S; ++c)
#pragma unroll
        for (int m = 0; m < V; ++m) sp[(long long)c * g.Nspec + l + LN * m] = v[c][m];
}

// ||out||^2 of out = scale F^-1{P : F[sigma]} without the inverse
// transforms (2D, S = 3): by Parseval the sum over the voxels of |out|^2 is
// scale^2 / N times the sum over all frequencies of |P : sigma^|^2, and the
// half spectrum (k_x in [0, n_x/2]) stands for k_x and n_x - k_x at once:
// weight 1 at k_x = 0 and, for even n_x, at k_x = n_x/2, else 2.  The
// forward y FFT and the projection are those of k_axis_wave; the spectrum is
// not written back.  Exactly nparts blocks per slot (the partial-sum layout
// of the x-inverse pass this replaces), each taking line positions in a
// grid-stride loop, so the sums are in a fixed order.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_axis_wave_norm(AxisArgs<T> a) {
    using WP = WavePlan<N>;
    constexpr int S = 3, V = WP::V, LN = WP::LN, LPW = 64 / LN;
    extern __shared__ unsigned char smem_raw[];
    const Geom& g = a.g;
    const int b = blockIdx.z;
    if (a.active && !a.active[b]) return;
    const int lane = threadIdx.x & 63, l = lane & (LN - 1), gl = lane / LN;
    const int wv = threadIdx.x >> 6, W = blockDim.x >> 6;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw) + (wv * LPW + gl) * lds_line(N);
    const cplx<T>* spb = a.spec + (long long)b * S * g.Nspec;
    const long long nlines = (long long)g.nxh * g.nz;
    cplx<T> wtw[WP::NTW];
    wave_twiddles<T, N>(a.tw, l, wtw);
    const T rN[3] = {T(1) / T(g.nx), T(1) / T(g.ny), T(1) / T(g.nz)};
    double acc = 0.0;
    for (long long base = ((long long)blockIdx.x * W + wv) * LPW; base < nlines;
         base += (long long)gridDim.x * W * LPW) {
        const long long L = base + gl;                // kx * nz + z
        if (L >= nlines) continue;                    // no barrier inside the loop
        const cplx<T>* sp = spb + L * N;
        cplx<T> v[S][V];
#pragma unroll
        for (int c = 0; c < S; ++c)
#pragma unroll
            for (int m = 0; m < V; ++m) v[c][m] = sp[(long long)c * g.Nspec + l + LN * m];
#pragma unroll
        for (int c = 0; c < S; ++c) wave_line_fft<T, N>(v[c], wtw, lds, l, false);
        const int kx = (int)(L / g.nz), kz = (int)(L - (long long)kx * g.nz);
        const double wgt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
        double line = 0.0;
#pragma unroll
        for (int m = 0; m < V; ++m) {
            T fx[3], fy[3];
            freq_xy<T>(g, kx, l + LN * m, kz, rN, fx, fy);
            cplx<T> u[S];
#pragma unroll
            for (int c = 0; c < S; ++c) u[c] = v[c][m];
            project2<T>(u, fx, fy);
#pragma unroll
            for (int c = 0; c < S; ++c) line += double(u[c].x) * double(u[c].x) + double(u[c].y) * double(u[c].y);
        }
        acc += wgt * line;
    }
    double pv[1] = {acc * a.nscale};
    block_sum_store<1>(pv, a.partials + (long long)b * a.nparts, 0, blockIdx.x);
}

// ---------------------------------------------------------------------------
// x-inverse pass
// ---------------------------------------------------------------------------

template <typename T, int S, int MODE, typename F, bool NT>
__global__ void __launch_bounds__(256) k_xinv(XinvArgs<T> a) {
    constexpr bool RT = x_reg_twiddles<F>();
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* const twl = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* buf = twl + (RT ? 0 : tw_lds_len<F>());
    const cplx<T>* const twp = (F::fast && !RT) ? twl : a.tw;
    const Geom& g = a.g;
    const int b = blockIdx.y;
    if (MODE == XI_CG) {
        if (a.cg[b].conv <= a.iter) return;
    } else if (MODE == XI_PCG) {
        if (a.pcg[b].conv <= a.iter) return;
    } else if (a.active && !a.active[b]) {
        return;
    }
    // CG: alpha = rr_k / p.Ap from the partials of the x-forward pass
    T alpha = T(0);
    if (MODE == XI_CG && a.cg[b].max_it >= 0) {
        double pap[1];
        block_sum_all<1>(a.pAp_part + (long long)b * a.nblocks, 0, a.nblocks, pap);
        if (!(pap[0] > 0.0) || !isfinite(pap[0])) {
            if (threadIdx.x == 0) {
                a.cg[b].status = 2;
                a.cg[b].conv = a.iter;
            }
            return;
        }
        alpha = T(a.cg[b].rr_hist[a.iter & 1] / pap[0]);
    }
    const int nx = line_len<F>(a.pl), nxh = nx / 2 + 1, ny = g.ny, nz = g.nz;
    const int nrows = ny * nz;
    const int RB = a.rows_per_block;          // a power of two
    const int npairs = RB / 2;
    const int lgp = __builtin_ctz(npairs);
    const int grp = xcd_group(blockIdx.x, gridDim.x);
    const int r0 = grp * RB;
    const int LS = lds_line(nx);
    const cplx<T>* sp = a.spec + (long long)b * S * g.Nspec;

    cplx<T> wr[RegTwCount<F>::n];
    if constexpr (RT) load_reg_twiddles<T, F::N>(a.tw, wr);
    else stage_twiddles<T, F>(twl, a.tw);     // ordered by the barrier before the FFT
    // gather Z = A + iB from the transposed half spectra of the row pair,
    // kLd elements per thread in flight before their LDS writes.  Each
    // half-spectrum value k is read once and gives Z_k = A_k + i B_k and,
    // for 0 < k < n_x/2, Z_{n_x-k} = conj(A_k) + i conj(B_k).  With an even
    // row count, rows 2i and 2i+1 of a frequency are adjacent and 16-byte
    // aligned, so in FP32 the pair is one load.
    const int gtot = S * npairs * nxh;
    const bool pair16 = sizeof(T) == 4 && (nrows & 1) == 0;
    for (int e0 = threadIdx.x; e0 < gtot; e0 += kLd * blockDim.x) {
        cplx<T> A[kLd], B[kLd];
        bool ina[kLd], inb[kLd];
#pragma unroll
        for (int u = 0; u < kLd; ++u) {     // unconditional loads at clamped addresses
            const int e = e0 + u * blockDim.x;
            const int pr = e & (npairs - 1);
            const int q = e >> lgp;               // q = c * nxh + k
            const int c = q / nxh;
            const int k = q - c * nxh;
            const int rowA = r0 + 2 * pr;
            const long long o = (long long)c * g.Nspec + (long long)k * nz * ny + rowA;
            ina[u] = e < gtot && rowA < nrows;
            inb[u] = e < gtot && rowA + 1 < nrows;
            if (pair16) ld_pair(sp + (ina[u] ? o : 0), A[u], B[u]);
            else {
                A[u] = sp[ina[u] ? o : 0];
                B[u] = sp[inb[u] ? o + 1 : 0];
            }
        }
        loads_issued();
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
            const int e = e0 + u * blockDim.x;
            if (e >= gtot) break;
            const int pr = e & (npairs - 1);
            const int q = e >> lgp;
            const int c = q / nxh;
            const int k = q - c * nxh;
            const T ax = ina[u] ? A[u].x : T(0), bx = inb[u] ? B[u].x : T(0);
            const T ay = ina[u] ? A[u].y : T(0), by = inb[u] ? B[u].y : T(0);
            cplx<T>* L = buf + (c * npairs + pr) * LS;
            L[lp(k)] = {ax - by, ay + bx};
            if (k > 0 && 2 * k < nx) L[lp(nx - k)] = {ax + by, bx - ay};
        }
    }
    __syncthreads();
    if constexpr (RT) line_fft_rt<T, F>(buf, S * npairs, LS, a.pl, wr, twp, true);
    else line_fft<T, F>(buf, S * npairs, LS, a.pl, twp, true);

    const T scale = T(g.inv_N) * a.scale;
    const long long fo = (long long)b * S * g.N;
    // loads of U voxels per thread ahead of their stores, as in k_xfwd
    constexpr int U = S == 6 ? 2 : 4;
    const int tot = RB * nx;
    double part = 0.0;
    for (int v0 = threadIdx.x; v0 < tot; v0 += U * blockDim.x) {
        T l0[U][S], l1[U][S];
        if constexpr (MODE != XI_STORE) {
#pragma unroll
            for (int u = 0; u < U; ++u) {       // unconditional, clamped addresses
                const int v = v0 + u * blockDim.x;
                const int rl = v / nx, x = v - rl * nx;
                const int row = r0 + rl;
                const long long idx = (long long)(v < tot && row < nrows ? row : 0) * nx + x;
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const long long o = fo + c * g.N + idx;
                    l0[u][c] = ld_s<NT>(a.r + o);
                    if constexpr (MODE == XI_PCG) l1[u][c] = a.sc[o];
                }
            }
            loads_issued();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * blockDim.x;
            const int rl = v / nx, x = v - rl * nx;
            const int row = r0 + rl;
            if (v >= tot || row >= nrows) continue;
            const long long idx = (long long)row * nx + x;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                const cplx<T> z = buf[(c * npairs + (rl >> 1)) * LS + lp(x)];
                const T q = ((rl & 1) ? z.y : z.x) * scale;
                const long long o = fo + c * g.N + idx;
                if constexpr (MODE == XI_STORE) {
                    if (a.out) a.out[o] = q;
                    part += double(q) * double(q);
                } else if constexpr (MODE == XI_PCG) {   // z = sc F^-1[...]; r.z
                    const T zz = l1[u][c] * q;
                    a.out[o] = zz;
                    part += double(l0[u][c]) * double(zz);
                } else {  // XI_CG (x takes alpha p in the next x-forward pass)
                    const T rn = l0[u][c] - alpha * q;
                    st_s<NT>(a.r + o, rn);
                    part += double(rn) * double(rn);
                }
            }
        }
    }
    double pv[1] = {part};
    block_sum_store<1>(pv, a.partials + (long long)b * a.nblocks, 0, grp);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

template <typename K, typename A>
static hipError_t launch_k(K kern, dim3 grid, size_t lds, hipStream_t st, const A& a) {
    hipLaunchKernelGGL(kern, grid, dim3(a.threads), lds, st, a);
    return hipGetLastError();
}

// Instantiate kernel template KT<T, S, MODE, F, NTV> for the FFT policy of
// the plan: fixed power-of-two length, else the runtime plan with maxb.
#define MIRVE_DISPATCH(KT, T, S, MODE, NTV, pl, maxb, grid, lds, st, a)                         \
    do {                                                                                         \
        switch ((pl).fastN) {                                                                    \
            case 16: return launch_k(KT<T, S, MODE, FastFFT<16>, NTV>, grid, lds, st, a);        \
            case 32: return launch_k(KT<T, S, MODE, FastFFT<32>, NTV>, grid, lds, st, a);        \
            case 64: return launch_k(KT<T, S, MODE, FastFFT<64>, NTV>, grid, lds, st, a);        \
            case 128: return launch_k(KT<T, S, MODE, FastFFT<128>, NTV>, grid, lds, st, a);      \
            case 256: return launch_k(KT<T, S, MODE, FastFFT<256>, NTV>, grid, lds, st, a);      \
            case 512: return launch_k(KT<T, S, MODE, FastFFT<512>, NTV>, grid, lds, st, a);      \
            case 1024: return launch_k(KT<T, S, MODE, FastFFT<1024>, NTV>, grid, lds, st, a);    \
            default: break;                                                                      \
        }                                                                                        \
        switch (maxb) {                                                                          \
            case 1: return launch_k(KT<T, S, MODE, GenericFFT<1>, NTV>, grid, lds, st, a);       \
            case 2: return launch_k(KT<T, S, MODE, GenericFFT<2>, NTV>, grid, lds, st, a);       \
            case 4: return launch_k(KT<T, S, MODE, GenericFFT<4>, NTV>, grid, lds, st, a);       \
            default: return launch_k(KT<T, S, MODE, GenericFFT<8>, NTV>, grid, lds, st, a);      \
        }                                                                                        \
    } while (0)

template <typename T, int S, int MODE, bool NT = false>
static hipError_t launch_xfwd_s(const XfwdArgs<T>& a, int maxb, size_t lds, hipStream_t st) {
    const dim3 grid(a.nblocks, a.g.B);
    MIRVE_DISPATCH(k_xfwd, T, S, MODE, NT, a.pl, maxb, grid, lds, st, a);
}

// Krylov modes with a.nt set stream their voxel vectors non-temporally.
template <typename T, int S, int MODE>
static hipError_t launch_xfwd_k(const XfwdArgs<T>& a, int maxb, size_t lds, hipStream_t st) {
    return a.nt ? launch_xfwd_s<T, S, MODE, true>(a, maxb, lds, st)
                : launch_xfwd_s<T, S, MODE, false>(a, maxb, lds, st);
}

template <typename T>
hipError_t launch_xfwd(const XfwdArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st) {
    if (mode == XF_PCG) return launch_xfwd_k<T, 1, XF_PCG>(a, maxb, lds, st);
    if (mode == XF_PCG0) return launch_xfwd_k<T, 1, XF_PCG0>(a, maxb, lds, st);
    if (a.g.s == 3) {
        switch (mode) {
            case XF_GREEN: return launch_xfwd_s<T, 3, XF_GREEN>(a, maxb, lds, st);
            case XF_CG: return launch_xfwd_k<T, 3, XF_CG>(a, maxb, lds, st);
            case XF_SPLIT: return launch_xfwd_s<T, 3, XF_SPLIT>(a, maxb, lds, st);
            case XF_CG_T: return launch_xfwd_k<T, 3, XF_CG_T>(a, maxb, lds, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (mode) {
        case XF_GREEN: return launch_xfwd_s<T, 6, XF_GREEN>(a, maxb, lds, st);
        case XF_CG: return launch_xfwd_k<T, 6, XF_CG>(a, maxb, lds, st);
        case XF_SPLIT: return launch_xfwd_s<T, 6, XF_SPLIT>(a, maxb, lds, st);
        case XF_CG_T: return launch_xfwd_k<T, 6, XF_CG_T>(a, maxb, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int S, int MODE>
static hipError_t launch_axis_s(const AxisArgs<T>& a, int maxb, dim3 grid, size_t lds,
                                hipStream_t st) {
    MIRVE_DISPATCH(k_axis, T, S, MODE, false, a.pl, maxb, grid, lds, st, a);
}

// Contiguous lines of 128, 256 or 512 points go to the one-wave pass (grid,
// block and LDS of its own) unless the handle keeps the block pass.
template <typename T, int S, int MODE>
static hipError_t launch_axis_wave(const AxisArgs<T>& a, hipStream_t st) {
    constexpr int W = 4;                       // waves per block
    const int N = a.g.ny;
    const int lpw = N >= 256 ? 1 : 2;          // lines per wave
    const long long nlines = (long long)a.g.nxh * a.g.nz;
    const long long waves = (nlines + lpw - 1) / lpw;
    const dim3 grid((unsigned)((waves + W - 1) / W), 1, a.g.B);
    const size_t lds = (size_t)W * lpw * lds_line(N) * sizeof(cplx<T>);
    if (N == 512) hipLaunchKernelGGL((k_axis_wave<T, S, MODE, 512>), grid, dim3(64 * W), lds, st, a);
    else if (N == 256) hipLaunchKernelGGL((k_axis_wave<T, S, MODE, 256>), grid, dim3(64 * W), lds, st, a);
    else hipLaunchKernelGGL((k_axis_wave<T, S, MODE, 128>), grid, dim3(64 * W), lds, st, a);
    return hipGetLastError();
}

// The norm pass: nparts blocks per slot (see k_axis_wave_norm).
template <typename T>
hipError_t launch_axis_norm(const AxisArgs<T>& a, hipStream_t st) {
    constexpr int W = 4;
    const int N = a.g.ny;
    if (a.contiguous == 0 || a.g.s != 3 || a.pl.N != N || a.nparts < 1 ||
        !(N == 128 || N == 256 || N == 512))
        return hipErrorInvalidValue;
    const int lpw = N >= 256 ? 1 : 2;
    const dim3 grid((unsigned)a.nparts, 1, a.g.B);
    const size_t lds = (size_t)W * lpw * lds_line(N) * sizeof(cplx<T>);
    if (N == 512) hipLaunchKernelGGL((k_axis_wave_norm<T, 512>), grid, dim3(64 * W), lds, st, a);
    else if (N == 256) hipLaunchKernelGGL((k_axis_wave_norm<T, 256>), grid, dim3(64 * W), lds, st, a);
    else hipLaunchKernelGGL((k_axis_wave_norm<T, 128>), grid, dim3(64 * W), lds, st, a);
    return hipGetLastError();
}

template <typename T>
static bool wave_axis_applies(const AxisArgs<T>& a) {
    return !a.block_only && a.contiguous && a.pl.N == a.g.ny &&
           (a.g.ny == 128 || a.g.ny == 256 || a.g.ny == 512);
}

// The damage preconditioner (a.pcg set) transforms one scalar field.
template <typename T>
hipError_t launch_axis(const AxisArgs<T>& a, int mode, int maxb, dim3 grid, size_t lds,
                       hipStream_t st) {
    if (wave_axis_applies(a)) {
        if (a.pcg) {
            switch (mode) {
                case AX_FWD: return launch_axis_wave<T, 1, AX_FWD>(a, st);
                case AX_INV: return launch_axis_wave<T, 1, AX_INV>(a, st);
                case AX_FWD_M_INV: return launch_axis_wave<T, 1, AX_FWD_M_INV>(a, st);
                default: break;
            }
        } else if (a.g.s == 3 && mode == AX_FWD_P_INV) {
            return launch_axis_wave<T, 3, AX_FWD_P_INV>(a, st);
        } else if (a.g.s == 6 && (mode == AX_FWD || mode == AX_INV)) {
            return mode == AX_FWD ? launch_axis_wave<T, 6, AX_FWD>(a, st)
                                  : launch_axis_wave<T, 6, AX_INV>(a, st);
        }
    }
    if (a.pcg) {
        switch (mode) {
            case AX_FWD: return launch_axis_s<T, 1, AX_FWD>(a, maxb, grid, lds, st);
            case AX_INV: return launch_axis_s<T, 1, AX_INV>(a, maxb, grid, lds, st);
            case AX_FWD_M_INV: return launch_axis_s<T, 1, AX_FWD_M_INV>(a, maxb, grid, lds, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.g.s == 3) {
        switch (mode) {
            case AX_FWD: return launch_axis_s<T, 3, AX_FWD>(a, maxb, grid, lds, st);
            case AX_INV: return launch_axis_s<T, 3, AX_INV>(a, maxb, grid, lds, st);
            case AX_FWD_P_INV: return launch_axis_s<T, 3, AX_FWD_P_INV>(a, maxb, grid, lds, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (mode) {
        case AX_FWD: return launch_axis_s<T, 6, AX_FWD>(a, maxb, grid, lds, st);
        case AX_INV: return launch_axis_s<T, 6, AX_INV>(a, maxb, grid, lds, st);
        case AX_FWD_P_INV: return launch_axis_s<T, 6, AX_FWD_P_INV>(a, maxb, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int S, int MODE, bool NT = false>
static hipError_t launch_xinv_s(const XinvArgs<T>& a, int maxb, size_t lds, hipStream_t st) {
    const dim3 grid(a.nblocks, a.g.B);
    MIRVE_DISPATCH(k_xinv, T, S, MODE, NT, a.pl, maxb, grid, lds, st, a);
}

template <typename T, int S, int MODE>
static hipError_t launch_xinv_k(const XinvArgs<T>& a, int maxb, size_t lds, hipStream_t st) {
    return a.nt ? launch_xinv_s<T, S, MODE, true>(a, maxb, lds, st)
                : launch_xinv_s<T, S, MODE, false>(a, maxb, lds, st);
}

template <typename T>
hipError_t launch_xinv(const XinvArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st) {
    if (mode == XI_PCG) return launch_xinv_k<T, 1, XI_PCG>(a, maxb, lds, st);
    if (a.g.s == 3)
        return mode == XI_CG ? launch_xinv_k<T, 3, XI_CG>(a, maxb, lds, st)
                             : launch_xinv_s<T, 3, XI_STORE>(a, maxb, lds, st);
    return mode == XI_CG ? launch_xinv_k<T, 6, XI_CG>(a, maxb, lds, st)
                         : launch_xinv_s<T, 6, XI_STORE>(a, maxb, lds, st);
}

// One object per precision (MIRVE_REAL = double or float) keeps the build parallel.
template hipError_t launch_xfwd<MIRVE_REAL>(const XfwdArgs<MIRVE_REAL>&, int, int, size_t, hipStream_t);
template hipError_t launch_axis<MIRVE_REAL>(const AxisArgs<MIRVE_REAL>&, int, int, dim3, size_t,
                                            hipStream_t);
template hipError_t launch_xinv<MIRVE_REAL>(const XinvArgs<MIRVE_REAL>&, int, int, size_t, hipStream_t);
template hipError_t launch_axis_norm<MIRVE_REAL>(const AxisArgs<MIRVE_REAL>&, hipStream_t);

}  // namespace mirve
