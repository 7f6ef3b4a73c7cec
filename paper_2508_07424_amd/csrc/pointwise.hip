// Pointwise and stencil kernels: unit response, history, the damage
// operator and the stencil steps of its preconditioned CG, the AT2
// functionals, the crack-tip enrichment energy, Anderson mixing, fracture
// test and the start-up kernels of the device-side Krylov scalars.
//
// Damage derivatives are forward differences with periodic wrap; the
// operator L(phi) = -div(G_c l grad phi) (Eq. 10b, 17) is D^T diag(G_c l) D,
// evaluated as a 2d+1 point stencil instead of the paper's FFT form (the two
// are the same linear map).
//
// Batches: blockIdx.y is the RVE; reductions write per-block partial sums to
// partials[(b * kMaxVals + v) * kRedBlocks + block], which a one-block-per-RVE
// kernel, or the next iteration's kernel itself, adds in a fixed order.
#include <cfloat>
#include "kernels.h"
#include "reduce.h"

namespace mirve {

constexpr int TPB = 256;

static inline int blocks_for(long long n) {
    long long b = (n + TPB - 1) / TPB;
    return (int)(b < 1 ? 1 : b);
}

__device__ inline double* pslot(double* partials, int b, int v) {
    return partials + ((long long)b * kMaxVals + v) * kRedBlocks;
}

__device__ inline bool skip(const int* active, int b) { return active && !active[b]; }

template <typename T>
__device__ inline T degr(T phi, T k) {
    const T u = T(1) - phi;
    return u * u + k;
}

struct Nb {
    long long xm, xp, ym, yp, zm, zp;
};

// q = u / d and u - q d in 32-bit arithmetic (a shift and a mask for a
// power-of-two d, uniform across the wave).
__device__ __forceinline__ unsigned divmod_u32(unsigned u, unsigned d, unsigned& r) {
    if ((d & (d - 1)) == 0) {
        r = u & (d - 1);
        return u >> __builtin_ctz(d);
    }
    const unsigned q = u / d;
    r = u - q * d;
    return q;
}

// Periodic neighbour indices of voxel idx of one RVE (N <= 2^30: every
// axis has at most 1024 voxels).
__device__ inline Nb neighbours(const Geom& g, long long idx) {
    unsigned x, y;
    const unsigned t = divmod_u32((unsigned)idx, (unsigned)g.nx, x);
    const unsigned z = divmod_u32(t, (unsigned)g.ny, y);
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    Nb n;
    n.xm = idx + (x == 0 ? g.nx - 1 : -1);
    n.xp = idx + (x == (unsigned)g.nx - 1 ? -(g.nx - 1) : 1);
    n.ym = idx + (y == 0 ? (g.ny - 1) * sy : -sy);
    n.yp = idx + (y == (unsigned)g.ny - 1 ? -(g.ny - 1) * sy : sy);
    n.zm = idx + (z == 0 ? (g.nz - 1) * sz : -sz);
    n.zp = idx + (z == (unsigned)g.nz - 1 ? -(g.nz - 1) * sz : sz);
    return n;
}

// ---------------------------------------------------------------------------
// cleavage anisotropy (Sec. 2.2, Eq. 14-17): the damage operator
// sum_jk D_j^T (w A_jk D_k p), A per voxel, forward differences D
// ---------------------------------------------------------------------------

// A_jk of a material entry (A stored as xx, yy, zz, yz, xz, xy)
template <typename T>
__device__ __forceinline__ T acoef(const MatEntry<T>& m, int j, int k) {
    if (j == k) return m.A[j];
    const int t = j + k;                       // (x, y) 1, (x, z) 2, (y, z) 3
    return m.A[t == 1 ? 5 : t == 2 ? 4 : 3];
}

// voxel idx shifted by (dx, dy, dz) voxels, periodic (|d| <= 1)
__device__ inline long long shifted(const Geom& g, long long idx, int dx, int dy, int dz) {
    unsigned xu, yu;
    const unsigned t = divmod_u32((unsigned)idx, (unsigned)g.nx, xu);
    const unsigned zu = divmod_u32(t, (unsigned)g.ny, yu);
    int x = (int)xu + dx, y = (int)yu + dy, z = (int)zu + dz;
    x += x < 0 ? g.nx : (x >= g.nx ? -g.nx : 0);
    y += y < 0 ? g.ny : (y >= g.ny ? -g.ny : 0);
    z += z < 0 ? g.nz : (z >= g.nz ? -g.nz : 0);
    return ((long long)z * g.ny + y) * g.nx + x;
}

__device__ __forceinline__ long long step_axis(const Geom& g, long long idx, int axis, int d) {
    return shifted(g, idx, axis == 0 ? d : 0, axis == 1 ? d : 0, axis == 2 ? d : 0);
}

// sum_j [w_j(i - e_j) - w_j(i)] h^-2 with w_j(k) = coef(k) sum_m A_jm(k)
// (p(k + e_m) - p(k)): the anisotropic part of the operator at voxel i.
// coef(k) is Gc(k) l (mode 0) or c (mode 1); pv(k) returns p at voxel k.
template <typename R, typename T, typename PV>
__device__ inline R aniso_div(const Geom& g, const uint16_t* mid, const MatEntry<T>* mt, int mode,
                              R c, long long i, PV pv) {
    const R ell = R(g.ell);
    const int d = g.dim;
    const R pi = pv(i);
    R acc = R(0);
    const MatEntry<T>& mi = mt[mid[i]];
    const R ci = mode == 0 ? R(mi.Gc) * ell : c;
    for (int j = 0; j < d; ++j) {
        // w_j at the voxel itself
        R wi = R(0);
        for (int m = 0; m < d; ++m) wi += R(acoef(mi, j, m)) * (pv(step_axis(g, i, m, 1)) - pi);
        // w_j at i - e_j, whose forward neighbour along j is i
        const long long k = step_axis(g, i, j, -1);
        const MatEntry<T>& mk = mt[mid[k]];
        const R ck = mode == 0 ? R(mk.Gc) * ell : c;
        const R pk = pv(k);
        R wk = R(0);
        for (int m = 0; m < d; ++m) {
            const long long km = m == j ? i : step_axis(g, k, m, 1);
            wk += R(acoef(mk, j, m)) * (pv(km) - pk);
        }
        acc += ck * wk - ci * wi;
    }
    return acc * R(1.0 / (g.h * g.h));
}

// grad a . A grad b at voxel i (forward differences, A of the voxel's entry)
template <typename R, typename T, typename PA, typename PB>
__device__ inline R aniso_grad_dot(const Geom& g, const MatEntry<T>& m, long long i, PA pa, PB pb) {
    const int d = g.dim;
    R ga[3], gb[3];
    const R a0 = pa(i), b0 = pb(i);
    for (int j = 0; j < d; ++j) {
        const long long nb = step_axis(g, i, j, 1);
        ga[j] = pa(nb) - a0;
        gb[j] = pb(nb) - b0;
    }
    R s = R(0);
    for (int j = 0; j < d; ++j)
        for (int k = 0; k < d; ++k) s += R(acoef(m, j, k)) * ga[j] * gb[k];
    return s * R(1.0 / (g.h * g.h));
}

// ---------------------------------------------------------------------------
// finalize kernels: one block of 256 threads per RVE (blockIdx.x = b)
// ---------------------------------------------------------------------------

// Fixed-order sum of n values: thread t adds entries t, t+256, ... in order,
// then a fixed tree over the threads.  Every thread returns the total.
__device__ inline double sum_fixed(const double* p, int n) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double tot = sh[0];
    __syncthreads();
    return tot;
}

__device__ inline double max_fixed(const double* p, int n) {
    __shared__ double sh[256];
    double s = -DBL_MAX;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s = fmax(s, p[i]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    const double tot = sh[0];
    __syncthreads();
    return tot;
}

__global__ void k_cg_init(CgDev* cgs, const double* prr, const double* pb, int n, double tol,
                          int max_it, const int* active) {
    const int b = blockIdx.x;
    CgDev* cg = cgs + b;
    if (skip(active, b)) {
        if (threadIdx.x == 0) { cg->conv = -1; cg->status = 0; }
        return;
    }
    const double rr = sum_fixed(prr + (long long)b * n, n);
    const double bn2 = sum_fixed(pb + (long long)b * n, n);
    if (threadIdx.x != 0) return;
    cg->rr_hist[0] = rr;
    cg->rr_hist[1] = rr;
    cg->rr = rr;
    cg->rr0 = rr;
    cg->bn2 = bn2;
    cg->tol2 = tol * tol;
    cg->max_it = max_it;
    cg->status = 0;
    cg->conv = kNotDone;
    if (!isfinite(rr) || !isfinite(bn2)) { cg->conv = 0; cg->status = 2; }
    else if (rr <= cg->tol2 * bn2) { cg->conv = 0; cg->status = 1; }
}

hipError_t launch_cg_init(CgDev* cg, const double* prr, const double* pb, int n, int B,
                          double tol, int max_it, const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init, dim3(B), dim3(256), 0, st, cg, prr, pb, n, tol, max_it, active);
    return hipGetLastError();
}
__global__ void k_sum_partials(const double* p, int n, int nv, double* sums, const int* active) {
    const int b = blockIdx.x;
    if (skip(active, b)) return;
    for (int v = 0; v < nv; ++v) {
        const double s = sum_fixed(p + ((long long)b * kMaxVals + v) * kRedBlocks, n);
        if (threadIdx.x == 0) sums[b * kMaxVals + v] = s;
    }
}
hipError_t launch_sum_partials(const double* p, int n, int nv, int B, double* sums,
                               const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(B), dim3(256), 0, st, p, n, nv, sums, active);
    return hipGetLastError();
}

__global__ void k_sum_rows(const double* p, int n, double* sums, int slot) {
    const int b = blockIdx.x;
    const double s = sum_fixed(p + (long long)b * n, n);
    if (threadIdx.x == 0) sums[b * kMaxVals + slot] = s;
}
hipError_t launch_sum_rows(const double* p, int n, int B, double* sums, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_rows, dim3(B), dim3(256), 0, st, p, n, sums, slot);
    return hipGetLastError();
}

__global__ void k_max_partials(const double* p, int n, double* sums, const int* active) {
    const int b = blockIdx.x;
    if (skip(active, b)) return;
    const double m = max_fixed(p + (long long)b * kMaxVals * kRedBlocks, n);
    if (threadIdx.x == 0) sums[b * kMaxVals] = m;
}
hipError_t launch_max_partials(const double* p, int n, int B, double* sums, const int* active,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_max_partials, dim3(B), dim3(256), 0, st, p, n, sums, active);
    return hipGetLastError();
}

__global__ void k_pcg_fin_start(PcgDev* ds, const double* p, int n, double tol, int max_it,
                                double inv_N, const int* active) {
    const int b = blockIdx.x;
    PcgDev* d = ds + b;
    if (skip(active, b)) {
        if (threadIdx.x == 0) { d->conv = -1; d->status = 0; }
        return;
    }
    const double* pb = p + (long long)b * kMaxVals * kRedBlocks;
    const double bn2 = sum_fixed(pb + 3 * kRedBlocks, n);
    const double asum = sum_fixed(pb + 4 * kRedBlocks, n);
    const double wsum = sum_fixed(pb + 5 * kRedBlocks, n);
    if (threadIdx.x != 0) return;
    d->bn2 = bn2;
    d->tol2 = tol * tol;
    d->abar = asum * inv_N;
    d->bbar = wsum * inv_N;
    d->max_it = max_it;
    d->status = 0;
    d->conv = kNotDone;
}
hipError_t launch_pcg_fin_start(PcgDev* d, const double* p, int n, int B, double tol, int max_it,
                                double inv_N, const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_fin_start, dim3(B), dim3(256), 0, st, d, p, n, tol, max_it, inv_N,
                       active);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// unit response and history
// ---------------------------------------------------------------------------

template <typename T, int S, bool SPLIT>
__global__ void __launch_bounds__(TPB) k_unit_response(Geom g, const uint16_t* mat_id,
                                                       const MatEntry<T>* mat, const T* phi,
                                                       const T* x, F6 f, T* psi1, T* eps1,
                                                       T* sig1, double* partials,
                                                       const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long so = (long long)b * g.N, fo = so * S;
    const MatEntry<T>* mt = mat + (long long)b * g.mstride;
    constexpr int NI = S == 3 ? 2 : 3;      // normal components (Mandel identity)
    double part = 0.0, part2 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const MatEntry<T>& m = mt[mat_id[so + i]];
        const T gg = degr(phi[so + i], T(g.k_res));
        T e[S], o[S];
#pragma unroll
        for (int c = 0; c < S; ++c) e[c] = T(f.v[c]) + x[fo + c * g.N + i];
        T psi = T(0);
#pragma unroll
        for (int a = 0; a < S; ++a) {
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < S; ++c) acc += m.C[a * S + c] * e[c];
            o[a] = acc;
            psi += e[a] * acc;
        }
        T sg[S];
#pragma unroll
        for (int c = 0; c < S; ++c) sg[c] = gg * o[c];
        if constexpr (SPLIT) {
            // sigma = g (C:e - K tr I + K <tr>+ I) + K <tr>- I; only the
            // tensile energy 1/2 e:C:e - 1/2 K tr^2 + 1/2 K <tr>+^2 drives damage
            T tr = T(0);
#pragma unroll
            for (int c = 0; c < NI; ++c) tr += e[c];
            const T add = tr > T(0) ? T(0) : (T(1) - gg) * m.K * tr;
#pragma unroll
            for (int c = 0; c < NI; ++c) sg[c] += add;
            psi -= tr > T(0) ? T(0) : m.K * tr * tr;
        }
        psi1[so + i] = T(0.5) * psi * m.drive;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            if (eps1) eps1[fo + c * g.N + i] = e[c];
            if (sig1) sig1[fo + c * g.N + i] = sg[c];
            part += double(sg[c]) * f.v[c];
            part2 += double(sg[c]) * double(sg[c]);
        }
    }
    double pv[2] = {part, part2};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_unit_response(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const T* phi, const T* x, const F6& f, int split, T* psi1,
                                T* eps1, T* sig1, double* partials, int nred, const int* active,
                                hipStream_t st) {
    const dim3 grid(nred, g.B);
    if (g.s == 3 && !split)
        hipLaunchKernelGGL((k_unit_response<T, 3, false>), grid, dim3(TPB), 0, st, g, mat_id, mat,
                           phi, x, f, psi1, eps1, sig1, partials, active);
    else if (g.s == 3)
        hipLaunchKernelGGL((k_unit_response<T, 3, true>), grid, dim3(TPB), 0, st, g, mat_id, mat,
                           phi, x, f, psi1, eps1, sig1, partials, active);
    else if (!split)
        hipLaunchKernelGGL((k_unit_response<T, 6, false>), grid, dim3(TPB), 0, st, g, mat_id, mat,
                           phi, x, f, psi1, eps1, sig1, partials, active);
    else
        hipLaunchKernelGGL((k_unit_response<T, 6, true>), grid, dim3(TPB), 0, st, g, mat_id, mat,
                           phi, x, f, psi1, eps1, sig1, partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_newton_update(Geom g, T* x, const T* dx, F6 f,
                                                       double* partials, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long fo = (long long)b * g.s * g.N;
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        for (int c = 0; c < g.s; ++c) {
            const long long o = fo + c * g.N + i;
            const T d = dx[o];
            const T xn = x[o] + d;
            x[o] = xn;
            const double e = double(xn) + f.v[c];
            s0 += double(d) * double(d);
            s1 += e * e;
        }
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_newton_update(const Geom& g, T* x, const T* dx, const F6& f, double* partials,
                                int nred, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_newton_update<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, x, dx, f,
                       partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_history(long long N, const T* psi1, const T* psi_ini,
                                                 const T* Hn, const double* E, int history, T* H,
                                                 T* rhs, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const long long o = (long long)b * N + i;
    const T E2 = T(E[b] * E[b]);
    const T ht = E2 * psi1[o] + psi_ini[o];
    const T h = history ? (ht > Hn[o] ? ht : Hn[o]) : ht;
    H[o] = h;
    if (rhs) rhs[o] = T(2) * h;
}

template <typename T>
hipError_t launch_history(const Geom& g, const T* psi1, const T* psi_ini, const T* Hn,
                          const double* E, int history, T* H, T* rhs, const int* active,
                          hipStream_t st) {
    hipLaunchKernelGGL((k_history<T>), dim3(blocks_for(g.N), g.B), dim3(TPB), 0, st, g.N, psi1,
                       psi_ini, Hn, E, history, H, rhs, active);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_commit_history(const Geom& g, const T* psi1, const T* psi_ini, const double* E,
                                 int history, T* Hn, const int* active, hipStream_t st) {
    // in place: Hn = max(E^2 psi1 + psi_ini, Hn)
    hipLaunchKernelGGL((k_history<T>), dim3(blocks_for(g.N), g.B), dim3(TPB), 0, st, g.N, psi1,
                       psi_ini, (const T*)Hn, E, history, Hn, (T*)nullptr, active);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// damage operator and its PCG
// ---------------------------------------------------------------------------

// a(x) and w(x) of the operator a p + D^T (w D p).
template <typename T>
__device__ inline void coeffs(const Geom& g, const MatEntry<T>* mat, const uint16_t* mid,
                              const T* H, int mode, T c, long long i, T& a, T& w) {
    if (mode == 0) {
        const T gc = mat[mid[i]].Gc;
        a = gc / T(g.ell) + (H ? T(2) * H[i] : T(0));
        w = gc * T(g.ell);
    } else {
        a = T(1);
        w = c;
    }
}

template <typename T>
__device__ inline T wcoef(const MatEntry<T>* mat, const uint16_t* mid, int mode, T ell, T c,
                          long long i) {
    return mode == 0 ? mat[mid[i]].Gc * ell : c;
}

// fields passed here are already offset to the RVE
template <typename T>
__device__ inline T apply_op(const Geom& g, const uint16_t* mid, const MatEntry<T>* mat,
                             const T* H, int mode, T c, const T* p, long long i) {
    T a, w;
    coeffs(g, mat, mid, H, mode, c, i, a, w);
    if (g.aniso)
        return a * p[i] + aniso_div<T>(g, mid, mat, mode, c, i, [&](long long k) { return p[k]; });
    const Nb n = neighbours(g, i);
    const T ell = T(g.ell);
    const T ih2 = T(1.0 / (g.h * g.h));
    const T pc = p[i];
    T acc = T(0);
    acc += wcoef(mat, mid, mode, ell, c, n.xm) * (pc - p[n.xm]) - w * (p[n.xp] - pc);
    acc += wcoef(mat, mid, mode, ell, c, n.ym) * (pc - p[n.ym]) - w * (p[n.yp] - pc);
    if (g.dim == 3)
        acc += wcoef(mat, mid, mode, ell, c, n.zm) * (pc - p[n.zm]) - w * (p[n.zp] - pc);
    return a * pc + acc * ih2;
}

#define RVE_OFFSETS                                                   \
    const long long so = (long long)b * g.N;                          \
    const uint16_t* mid = mat_id + so;                                \
    const MatEntry<T>* mt = mat + (long long)b * g.mstride;

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_matvec(Geom g, const uint16_t* mat_id,
                                                    const MatEntry<T>* mat, const T* H, int mode,
                                                    T c, const T* p, T* q, double* partials,
                                                    const PcgDev* d, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    if (d && d[b].conv != kNotDone) return;
    RVE_OFFSETS
    const T* Hb = H ? H + so : nullptr;
    double part = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const T v = apply_op(g, mid, mt, Hb, mode, c, p + so, i);
        q[so + i] = v;
        part += double(p[so + i]) * double(v);
    }
    if (partials) {
        double pv[1] = {part};
        block_sum_store<1>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
    }
}

template <typename T>
hipError_t launch_pcg_matvec(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, double c, const T* p, T* q, double* partials,
                             int nred, const PcgDev* d, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_matvec<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat, H,
                       mode, T(c), p, q, partials, d, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_damage_diag(Geom g, const uint16_t* mat_id,
                                                     const MatEntry<T>* mat, const T* H, int mode,
                                                     T c, int sqrt_out, T* dinv, double* partials,
                                                     const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const T* Hb = H ? H + so : (const T*)nullptr;
    const T ell = T(g.ell);
    double sa = 0.0, sw = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        T a, w;
        coeffs(g, mt, mid, Hb, mode, c, i, a, w);
        const Nb n = neighbours(g, i);
        T s;
        if (g.aniso) {
            // sum_j [coef(i - e_j) A_jj(i - e_j) + coef(i) sum_m A_jm(i)]
            s = T(0);
            const MatEntry<T>& mi = mt[mid[i]];
            for (int j = 0; j < g.dim; ++j) {
                const long long k = step_axis(g, i, j, -1);
                s += wcoef(mt, mid, mode, ell, c, k) * acoef(mt[mid[k]], j, j);
                for (int m = 0; m < g.dim; ++m) s += w * acoef(mi, j, m);
            }
        } else {
            s = T(2) * w + wcoef(mt, mid, mode, ell, c, n.xm) + wcoef(mt, mid, mode, ell, c, n.ym);
            if (g.dim == 3) s += w + wcoef(mt, mid, mode, ell, c, n.zm);
        }
        const T di = T(1) / (a + s * T(1.0 / (g.h * g.h)));
        dinv[so + i] = sqrt_out ? sqrt(di) : di;
        sa += double(a);
        sw += double(w);
    }
    double pv[2] = {sa, sw};
    block_sum_store<2>(pv, pslot(partials, b, 4), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_damage_diag(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* H, int mode, double c, int sqrt_out, T* dinv,
                              double* partials, int nred, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_damage_diag<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat, H,
                       mode, T(c), sqrt_out, dinv, partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_start(long long N, const T* bv, const T* Ax,
                                                   const T* dinv, T* r, double* partials,
                                                   const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long so = (long long)b * N;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const long long o = so + i;
        const T bi = bv[o];
        const T ri = bi - Ax[o];
        r[o] = ri;
        s0 += double(ri) * double(dinv[o] * ri);
        s1 += double(ri) * double(ri);
        s2 += double(bi) * double(bi);
    }
    double pv[3] = {s0, s1, s2};
    block_sum_store<3>(pv, pslot(partials, b, 1), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_pcg_start(const Geom& g, const T* b, const T* Ax, const T* dinv, T* r,
                            double* partials, int nred, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_start<T>), dim3(nred, g.B), dim3(TPB), 0, st, g.N, b, Ax, dinv, r,
                       partials, active);
    return hipGetLastError();
}

// z at any voxel: dinv r (Jacobi) or the stored preconditioned residual
template <typename T, int PRE>
__device__ __forceinline__ T zval(const T* r, const T* dinv, const T* zf, long long j) {
    if constexpr (PRE == PRE_JACOBI) return dinv[j] * r[j];
    else return zf[j];
}

// U voxels per thread and round of the direction update + operator below, in
// three phases: (1) the independent loads (phase ids, history, z and the old
// direction at the voxel and its 2 d neighbours), at clamped addresses so
// that none waits for another; (2) the Gc of the phase ids; (3) arithmetic
// and stores.  U = 2: a larger U holds more values in flight per thread but
// costs more in occupancy (measured slower at U = 4).  Returns the thread's
// p.q partial.
template <typename T, int PRE, int DIM, int U>
__device__ __forceinline__ double matvec_dir_rounds(const Geom& g, const uint16_t* mid,
                                                    const MatEntry<T>* mt, const T* Hb, int mode,
                                                    T c, const T* r, const T* dinv, const T* zf,
                                                    const T* po, T beta, bool first, T* pn, T* q) {
    constexpr int NP = 1 + 2 * DIM;       // the voxel, then xm, xp, ym, yp (zm, zp)
    constexpr int NW = 1 + DIM;           // Gc at the voxel and at xm, ym (zm)
    const T ell = T(g.ell);
    const T ih2 = T(1.0 / (g.h * g.h));
    const long long N = g.N;
    const long long stride = (long long)gridDim.x * blockDim.x;
    double part = 0.0;
    for (long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; i0 < N; i0 += U * stride) {
        T zz[U][NP], pp[U][NP], hh[U], gcw[U][NW];
        int id[U][NW];
        long long iv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + u * stride;
            iv[u] = i;
            const Nb n = neighbours(g, i < N ? i : 0);
            const long long j[7] = {i < N ? i : 0, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp};
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if constexpr (PRE == PRE_JACOBI) zz[u][k] = dinv[j[k]] * r[j[k]];
                else zz[u][k] = zf[j[k]];
                pp[u][k] = first ? T(0) : po[j[k]];
            }
            hh[u] = Hb ? Hb[j[0]] : T(0);
            if (mode == 0) {
                id[u][0] = mid[j[0]];
#pragma unroll
                for (int k = 1; k < NW; ++k) id[u][k] = mid[j[2 * k - 1]];
            }
        }
        loads_issued();
        if (mode == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < NW; ++k) gcw[u][k] = mt[id[u][k]].Gc;
            loads_issued();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (iv[u] >= N) break;
            T a, w, wm[NW];
            if (mode == 0) {
                a = gcw[u][0] / ell + (Hb ? T(2) * hh[u] : T(0));
                w = gcw[u][0] * ell;
#pragma unroll
                for (int k = 1; k < NW; ++k) wm[k] = gcw[u][k] * ell;
            } else {
                a = T(1);
                w = c;
#pragma unroll
                for (int k = 1; k < NW; ++k) wm[k] = c;
            }
            T pd[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) pd[k] = first ? zz[u][k] : zz[u][k] + beta * pp[u][k];
            const T pc = pd[0];
            T acc = T(0);
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                acc += wm[d + 1] * (pc - pd[1 + 2 * d]) - w * (pd[2 + 2 * d] - pc);
            const T v = a * pc + acc * ih2;
            pn[iv[u]] = pc;
            q[iv[u]] = v;
            part += double(pc) * double(v);
        }
    }
    return part;
}

// One PCG step: r.z and r.r of the residual left by the previous step and
// the stopping test; then p = z + beta p_old (p = z at k = 0, where p_old is
// not read: it may hold anything), q = A p and the p.q partials.
template <typename T, int PRE>
__global__ void __launch_bounds__(TPB) k_pcg_matvec_dir(
    Geom g, const uint16_t* mat_id, const MatEntry<T>* mat, const T* H, int mode, T c,
    const T* r_a, const T* dinv_a, const T* zf_a, const T* po_a, T* pn_a, T* q_a,
    const double* rz_part, long long rz_stride, int rz_n, const double* rr_part,
    long long rr_stride, int rr_n, double* partials, PcgDev* d, int k) {
    const int b = blockIdx.y;
    if (d[b].conv <= k) return;
    double rz[1], rr[1];
    block_sum_all<1>(rz_part + (long long)b * rz_stride, 0, rz_n, rz);
    block_sum_all<1>(rr_part + (long long)b * rr_stride, 0, rr_n, rr);
    int stop = 0;
    if (!isfinite(rr[0]) || !isfinite(rz[0])) stop = 2;
    else if (rr[0] <= d[b].tol2 * d[b].bn2 || d[b].bn2 == 0.0) stop = 1;   // b = 0: x = 0 (host)
    else if (k >= d[b].max_it) stop = 3;
    const double prev = k > 0 ? d[b].rz_hist[(k - 1) & 1] : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d[b].rz_hist[k & 1] = rz[0];
        d[b].rr = rr[0];
        if (k == 0) d[b].rr0 = rr[0];
        if (stop) {
            d[b].status = stop;
            d[b].conv = k;
        }
    }
    if (stop) return;
    const T beta = k > 0 ? T(rz[0] / prev) : T(0);
    RVE_OFFSETS
    const T* Hb = H ? H + so : nullptr;
    const T* zf = zf_a ? zf_a + so : nullptr;
    double part;
    if (g.aniso) {
        // the direction p = z + beta p_old formed at every voxel the
        // anisotropic stencil reads (the voxel, its axis and diagonal
        // neighbours), then q = A p
        const T* r = r_a + so;
        const T* dv = dinv_a + so;
        const T* po = po_a + so;
        const bool first = k == 0;
        auto pv = [&](long long j) {
            const T z = zval<T, PRE>(r, dv, zf, j);
            return first ? z : z + beta * po[j];
        };
        part = 0.0;
        for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
             i += (long long)gridDim.x * blockDim.x) {
            T a, w;
            coeffs(g, mt, mid, Hb, mode, c, i, a, w);
            const T pc = pv(i);
            const T v = a * pc + aniso_div<T>(g, mid, mt, mode, c, i, pv);
            pn_a[so + i] = pc;
            q_a[so + i] = v;
            part += double(pc) * double(v);
        }
    } else if (g.dim == 2)
        part = matvec_dir_rounds<T, PRE, 2, 2>(g, mid, mt, Hb, mode, c, r_a + so, dinv_a + so, zf,
                                               po_a + so, beta, k == 0, pn_a + so, q_a + so);
    else
        part = matvec_dir_rounds<T, PRE, 3, 2>(g, mid, mt, Hb, mode, c, r_a + so, dinv_a + so, zf,
                                               po_a + so, beta, k == 0, pn_a + so, q_a + so);
    double pv[1] = {part};
    block_sum_store<1>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_pcg_matvec_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* H, int mode, double c, int pre, const T* r,
                                 const T* dinv, const T* zf, const T* p_old, T* p_new, T* q,
                                 const double* rz_part, long long rz_stride, int rz_n,
                                 const double* rr_part, long long rr_stride, int rr_n,
                                 double* partials, int nblk, PcgDev* d, int iter, hipStream_t st) {
    if (pre == PRE_JACOBI)
        hipLaunchKernelGGL((k_pcg_matvec_dir<T, PRE_JACOBI>), dim3(nblk, g.B), dim3(TPB), 0, st, g,
                           mat_id, mat, H, mode, T(c), r, dinv, zf, p_old, p_new, q, rz_part,
                           rz_stride, rz_n, rr_part, rr_stride, rr_n, partials, d, iter);
    else
        hipLaunchKernelGGL((k_pcg_matvec_dir<T, PRE_FFT>), dim3(nblk, g.B), dim3(TPB), 0, st, g,
                           mat_id, mat, H, mode, T(c), r, dinv, zf, p_old, p_new, q, rz_part,
                           rz_stride, rz_n, rr_part, rr_stride, rr_n, partials, d, iter);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_update(long long N, PcgDev* d, T* x, T* r,
                                                    const T* p, const T* q, const T* dinv,
                                                    double* partials, int n_pq, int k) {
    const int b = blockIdx.y;
    if (d[b].conv <= k) return;
    double pq[1];
    block_sum_all<1>(pslot(partials, b, 0), 0, n_pq, pq);
    if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            d[b].status = 2;
            d[b].conv = k;
        }
        return;
    }
    const T alpha = T(d[b].rz_hist[k & 1] / pq[0]);
    const long long so = (long long)b * N;
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const long long o = so + i;
        x[o] += alpha * p[o];
        const T ri = r[o] - alpha * q[o];
        r[o] = ri;
        s0 += double(ri) * double(dinv[o] * ri);
        s1 += double(ri) * double(ri);
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, pslot(partials, b, 1), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_pcg_update(const Geom& g, PcgDev* d, T* x, T* r, const T* p, const T* q,
                             const T* dinv, double* partials, int n_pq, int nred, int iter,
                             hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(nred, g.B), dim3(TPB), 0, st, g.N, d, x, r, p, q,
                       dinv, partials, n_pq, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AT2 functionals, residual, enrichment energy, tangent
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_dissipation(Geom g, const uint16_t* mat_id,
                                                     const MatEntry<T>* mat, const T* phi_all,
                                                     double* partials, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const T* phi = phi_all + so;
    double sD = 0.0, sG = 0.0;
    const double ell = g.ell, ih = 1.0 / g.h;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double pc = phi[i];
        double gag;
        if (g.aniso) {
            auto pv = [&](long long k) { return double(phi[k]); };
            gag = aniso_grad_dot<double>(g, mt[mid[i]], i, pv, pv);
        } else {
            const double gx = (double(phi[n.xp]) - pc) * ih;
            const double gy = (double(phi[n.yp]) - pc) * ih;
            const double gz = g.dim == 3 ? (double(phi[n.zp]) - pc) * ih : 0.0;
            gag = gx * gx + gy * gy + gz * gz;
        }
        const double dens = pc * pc / (2.0 * ell) + 0.5 * ell * gag;
        sD += double(mt[mid[i]].Gc) * dens;
        sG += dens;
    }
    double pv[2] = {sD, sG};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_dissipation(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* phi, double* partials, int nred, const int* active,
                              hipStream_t st) {
    hipLaunchKernelGGL((k_dissipation<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat, phi,
                       partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_damage_residual(Geom g, const uint16_t* mat_id,
                                                         const MatEntry<T>* mat, const T* H,
                                                         const T* phi, double* partials,
                                                         const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const T v = apply_op(g, mid, mt, H + so, 0, T(0), phi + so, i);
        const double bb = 2.0 * double(H[so + i]);
        const double res = double(v) - bb;
        s0 += res * res;
        s1 += bb * bb;
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_damage_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* H, const T* phi, double* partials, int nred,
                                  const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_damage_residual<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat,
                       H, phi, partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_psi_ini(Geom g, const uint16_t* mat_id,
                                                 const MatEntry<T>* mat, const T* phi,
                                                 T* psi_ini, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    RVE_OFFSETS
    // gamma'(phi) = Gc phi / l + L phi  (operator with H = 0)
    const T gp = apply_op(g, mid, mt, (const T*)nullptr, 0, T(0), phi + so, i);
    const T v = gp / (T(2) * (T(1) - phi[so + i]));
    psi_ini[so + i] = v > T(0) ? v : T(0);
}

template <typename T>
hipError_t launch_psi_ini(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                          const T* phi, T* psi_ini, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_psi_ini<T>), dim3(blocks_for(g.N), g.B), dim3(TPB), 0, st, g, mat_id,
                       mat, phi, psi_ini, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_tangent_rhs(long long N, const T* phi, const T* psi1,
                                                     const T* psi_ini, const T* Hn,
                                                     const double* E, int history, T* out,
                                                     const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const long long o = (long long)b * N + i;
    const T e = T(E[b]);
    const T ht = e * e * psi1[o] + psi_ini[o];
    const bool on = history ? (ht > Hn[o]) : true;
    out[o] = on ? T(2) * (T(1) - phi[o]) * T(2) * e * psi1[o] : T(0);
}

template <typename T>
hipError_t launch_tangent_rhs(const Geom& g, const T* phi, const T* psi1, const T* psi_ini,
                              const T* Hn, const double* E, int history, T* out,
                              const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_tangent_rhs<T>), dim3(blocks_for(g.N), g.B), dim3(TPB), 0, st, g.N, phi,
                       psi1, psi_ini, Hn, E, history, out, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_dissipation_dir(Geom g, const uint16_t* mat_id,
                                                         const MatEntry<T>* mat, const T* phi_a,
                                                         const T* dphi_a, double* partials,
                                                         const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const T* phi = phi_a + so;
    const T* dphi = dphi_a + so;
    double s = 0.0;
    const double ell = g.ell, ih = 1.0 / g.h;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double pc = phi[i], dc = dphi[i];
        double gg;
        if (g.aniso) {
            gg = aniso_grad_dot<double>(g, mt[mid[i]], i, [&](long long k) { return double(phi[k]); },
                                        [&](long long k) { return double(dphi[k]); }) / (ih * ih);
        } else {
            gg = (double(phi[n.xp]) - pc) * (double(dphi[n.xp]) - dc);
            gg += (double(phi[n.yp]) - pc) * (double(dphi[n.yp]) - dc);
            if (g.dim == 3) gg += (double(phi[n.zp]) - pc) * (double(dphi[n.zp]) - dc);
        }
        s += double(mt[mid[i]].Gc) * (pc * dc / ell + ell * gg * ih * ih);
    }
    double pv[1] = {s};
    block_sum_store<1>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_dissipation_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* phi, const T* dphi, double* partials, int nred,
                                  const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_dissipation_dir<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat,
                       phi, dphi, partials, active);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// field utilities (n elements per RVE)
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_copy(const T* s, T* d, long long n, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) d[(long long)b * n + i] = s[(long long)b * n + i];
}
template <typename T>
hipError_t launch_copy(const T* s, T* d, long long n, int B, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_copy<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, s, d, n, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_fill(T* d, T v, long long n, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) d[(long long)b * n + i] = v;
}
template <typename T>
hipError_t launch_fill(T* d, T v, long long n, int B, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, d, v, n, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_sub(const T* a, const T* c, T* out, long long n,
                                             const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) {
        const long long o = (long long)b * n + i;
        out[o] = a[o] - c[o];
    }
}
template <typename T>
hipError_t launch_sub(const T* a, const T* c, T* out, long long n, int B, const int* active,
                      hipStream_t st) {
    hipLaunchKernelGGL((k_sub<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, a, c, out, n, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_max_field(const T* a, long long n, double* partials,
                                                   const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    double m = -DBL_MAX;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        m = fmax(m, double(a[(long long)b * n + i]));
    block_max_store(m, pslot(partials, b, 0), blockIdx.x);
}
template <typename T>
hipError_t launch_max_field(const T* a, long long n, int B, double* partials, int nred,
                            const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_max_field<T>), dim3(nred, B), dim3(TPB), 0, st, a, n, partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_scale_field(T* a, const double* den, double c,
                                                     long long n, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) {
        const long long o = (long long)b * n + i;
        a[o] = T(double(a[o]) * (c / den[b * kMaxVals]));
    }
}
template <typename T>
hipError_t launch_scale_field(T* a, const double* den, double c, long long n, int B,
                              const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_field<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, a, den, c, n,
                       active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_diff_norms(const T* a, const T* c, long long n,
                                                    double* partials, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long o = (long long)b * n + i;
        const double d = double(a[o]) - double(c[o]);
        s0 += d * d;
        s1 += double(a[o]) * double(a[o]);
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}
template <typename T>
hipError_t launch_diff_norms(const T* a, const T* c, long long n, int B, double* partials,
                             int nred, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_diff_norms<T>), dim3(nred, B), dim3(TPB), 0, st, a, c, n, partials,
                       active);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Anderson mixing of the stagger iterates
// ---------------------------------------------------------------------------

template <typename T, int MM>
__global__ void __launch_bounds__(TPB) k_anderson_gram(long long N, const T* Fbase,
                                                       long long sstride, const int* order,
                                                       const int* m1a, double* partials,
                                                       const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const int m1 = m1a[b];
    const int m = m1 - 1;
    const T* F[MM + 1];
#pragma unroll
    for (int k = 0; k <= MM; ++k)
        F[k] = Fbase + (long long)order[b * kHist + (k < m1 ? k : 0)] * sstride + (long long)b * N;
    double acc[MM * MM + MM];
#pragma unroll
    for (int k = 0; k < MM * MM + MM; ++k) acc[k] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        double f[MM + 1];
#pragma unroll
        for (int k = 0; k <= MM; ++k) f[k] = k < m1 ? double(F[k][i]) : 0.0;
        double df[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) df[k] = k < m ? f[k + 1] - f[k] : 0.0;
        double last = 0.0;
#pragma unroll
        for (int k = 0; k <= MM; ++k)
            if (k == m) last = f[k];
#pragma unroll
        for (int a = 0; a < MM; ++a) {
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[a * MM + c] += df[a] * df[c];
            acc[MM * MM + a] += df[a] * last;
        }
    }
    block_sum_store<MM * MM + MM>(acc, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_anderson_gram(const Geom& g, const T* Fbase, long long slot_stride,
                                const int* order, const int* m1, double* partials, int nred,
                                const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_anderson_gram<T, kAndersonMax>), dim3(nred, g.B), dim3(TPB), 0, st, g.N,
                       Fbase, slot_stride, order, m1, partials, active);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_anderson_mix(long long N, const T* Gbase,
                                                      long long sstride, const int* order,
                                                      const int* m1a, const double* gamma, T* out,
                                                      const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int m = m1a[b] - 1;
    auto G = [&](int k) {
        return double(Gbase[(long long)order[b * kHist + k] * sstride + (long long)b * N + i]);
    };
    double v = G(m);
    for (int k = 0; k < m; ++k) v -= gamma[b * kAndersonMax + k] * (G(k + 1) - G(k));
    out[(long long)b * N + i] = T(v);
}

template <typename T>
hipError_t launch_anderson_mix(const Geom& g, const T* Gbase, long long slot_stride,
                               const int* order, const int* m1, const double* gamma, T* out,
                               const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_anderson_mix<T>), dim3(blocks_for(g.N), g.B), dim3(TPB), 0, st, g.N,
                       Gbase, slot_stride, order, m1, gamma, out, active);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fracture test: lines along the load axis without a broken voxel
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_fracture(Geom g, const uint16_t* mat_id,
                                                  const MatEntry<T>* mat, const T* phi_a, T thr,
                                                  int axis, int* count, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const T* phi = phi_a + so;
    const long long nlines = g.N / (axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz);
    const long long l = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    long long base, stride;
    int len;
    if (axis == 0) { base = l * g.nx; stride = 1; len = g.nx; }
    else if (axis == 1) {
        const long long x = l % g.nx, z = l / g.nx;
        base = z * (long long)g.nx * g.ny + x; stride = g.nx; len = g.ny;
    } else { base = l; stride = (long long)g.nx * g.ny; len = g.nz; }
    bool broken = false;
    for (int k = 0; k < len && !broken; ++k) {
        const long long i = base + k * stride;
        if (phi[i] >= thr || mt[mid[i]].drive == T(0)) broken = true;
    }
    if (!broken) atomicAdd(count + b, 1);
}

template <typename T>
hipError_t launch_fracture_count(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* phi, double thr, int axis, int* count,
                                 const int* active, hipStream_t st) {
    const long long nlines = g.N / (axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz);
    hipLaunchKernelGGL((k_fracture<T>), dim3(blocks_for(nlines), g.B), dim3(TPB), 0, st, g,
                       mat_id, mat, phi, T(thr), axis, count, active);
    return hipGetLastError();
}

__global__ void k_zero_int(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
hipError_t launch_zero_int(int* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_int, dim3(blocks_for(n)), dim3(TPB), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Iterative refinement of the damage balance (mixed precision).  The
// solution phi64 is held in FP64; the residual of the system with the bulk
// data (H, Gc in the bulk type) is formed in FP64 arithmetic, the correction
// comes from the bulk-precision PCG, and the update is FP64.
// ---------------------------------------------------------------------------

// r = 2H - A phi64 (Eq. 16b, mode 0 of apply_op) in FP64, stored in the bulk
// type for the correction solve; partials ||r||^2 and ||2H||^2.  The history
// field of load E, H = max(E^2 psi1 + psi_ini, H^n) (Eq. 38; without the max
// when history is off), is formed here in FP64 from the bulk-type fields, so
// that D(phi(E)) is a smooth function of E and not one quantised by the
// rounding of H to the bulk type.
template <typename T>
__global__ void __launch_bounds__(TPB) k_ir_residual(Geom g, const uint16_t* mat_id,
                                                     const MatEntry<T>* mat, const T* psi1,
                                                     const T* psi_ini, const T* Hn,
                                                     const double* E, int history,
                                                     const double* phi64, T* r, double* partials,
                                                     const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const double* p = phi64 + so;
    const double ell = g.ell, ih2 = 1.0 / (g.h * g.h), E2 = E[b] * E[b];
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double gc = double(mt[mid[i]].Gc);
        const double ht = E2 * double(psi1[so + i]) + double(psi_ini[so + i]);
        const double hn = double(Hn[so + i]);
        const double hb = 2.0 * (history && hn > ht ? hn : ht);
        const double a = gc / ell + hb, w = gc * ell, pc = p[i];
        double op;
        if (g.aniso) {
            op = a * pc + aniso_div<double>(g, mid, mt, 0, 0.0, i, [&](long long k) { return p[k]; });
        } else {
            double acc = double(mt[mid[n.xm]].Gc) * ell * (pc - p[n.xm]) - w * (p[n.xp] - pc);
            acc += double(mt[mid[n.ym]].Gc) * ell * (pc - p[n.ym]) - w * (p[n.yp] - pc);
            if (g.dim == 3) acc += double(mt[mid[n.zm]].Gc) * ell * (pc - p[n.zm]) - w * (p[n.zp] - pc);
            op = a * pc + acc * ih2;
        }
        const double res = hb - op;
        r[so + i] = T(res);
        s0 += res * res;
        s1 += hb * hb;
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_ir_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* psi1, const T* psi_ini, const T* Hn, const double* E,
                              int history, const double* phi64, T* r, double* partials, int nred,
                              const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_ir_residual<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat, psi1,
                       psi_ini, Hn, E, history, phi64, r, partials, active);
    return hipGetLastError();
}

// phi64 += delta; phi = phi64 rounded to the bulk type (delta may be null:
// rounding only)
template <typename T>
__global__ void __launch_bounds__(TPB) k_ir_update(double* phi64, const T* delta, T* phi, long long n,
                                                   const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long o = (long long)b * n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double v = phi64[o + i];
        if (delta) {
            v += double(delta[o + i]);
            phi64[o + i] = v;
        }
        if (phi) phi[o + i] = T(v);
    }
}

template <typename T>
hipError_t launch_ir_update(double* phi64, const T* delta, T* phi, long long n, int B,
                            const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_ir_update<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, phi64, delta,
                       phi, n, active);
    return hipGetLastError();
}

// phi64 = phi (widening copy)
template <typename T>
__global__ void __launch_bounds__(TPB) k_widen(const T* phi, double* phi64, long long n,
                                               const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    const long long o = (long long)b * n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        phi64[o + i] = double(phi[o + i]);
}

template <typename T>
hipError_t launch_widen(const T* phi, double* phi64, long long n, int B, const int* active,
                        hipStream_t st) {
    hipLaunchKernelGGL((k_widen<T>), dim3(blocks_for(n), B), dim3(TPB), 0, st, phi, phi64, n, active);
    return hipGetLastError();
}

// D and Gamma (Eq. 3, 4) of an FP64 damage field with the bulk material table
template <typename T>
__global__ void __launch_bounds__(TPB) k_dissipation64(Geom g, const uint16_t* mat_id,
                                                       const MatEntry<T>* mat, const double* phi_all,
                                                       double* partials, const int* active) {
    const int b = blockIdx.y;
    if (skip(active, b)) return;
    RVE_OFFSETS
    const double* phi = phi_all + so;
    double sD = 0.0, sG = 0.0;
    const double ell = g.ell, ih = 1.0 / g.h;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double pc = phi[i];
        double gag;
        if (g.aniso) {
            auto pv = [&](long long k) { return phi[k]; };
            gag = aniso_grad_dot<double>(g, mt[mid[i]], i, pv, pv);
        } else {
            const double gx = (phi[n.xp] - pc) * ih;
            const double gy = (phi[n.yp] - pc) * ih;
            const double gz = g.dim == 3 ? (phi[n.zp] - pc) * ih : 0.0;
            gag = gx * gx + gy * gy + gz * gz;
        }
        const double dens = pc * pc / (2.0 * ell) + 0.5 * ell * gag;
        sD += double(mt[mid[i]].Gc) * dens;
        sG += dens;
    }
    double pv[2] = {sD, sG};
    block_sum_store<2>(pv, pslot(partials, b, 0), kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_dissipation64(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const double* phi64, double* partials, int nred, const int* active,
                                hipStream_t st) {
    hipLaunchKernelGGL((k_dissipation64<T>), dim3(nred, g.B), dim3(TPB), 0, st, g, mat_id, mat,
                       phi64, partials, active);
    return hipGetLastError();
}

#define INST(T)                                                                                    \
    template hipError_t launch_ir_residual<T>(const Geom&, const uint16_t*, const MatEntry<T>*,    \
                                              const T*, const T*, const T*, const double*, int,    \
                                              const double*, T*, double*, int, const int*,         \
                                              hipStream_t);                                        \
    template hipError_t launch_ir_update<T>(double*, const T*, T*, long long, int, const int*,     \
                                            hipStream_t);                                          \
    template hipError_t launch_widen<T>(const T*, double*, long long, int, const int*,             \
                                        hipStream_t);                                              \
    template hipError_t launch_dissipation64<T>(const Geom&, const uint16_t*, const MatEntry<T>*,  \
                                                const double*, double*, int, const int*,           \
                                                hipStream_t);                                      \
    template hipError_t launch_unit_response<T>(const Geom&, const uint16_t*, const MatEntry<T>*,  \
                                                const T*, const T*, const F6&, int, T*, T*, T*,    \
                                                double*, int, const int*, hipStream_t);            \
    template hipError_t launch_newton_update<T>(const Geom&, T*, const T*, const F6&, double*,     \
                                                int, const int*, hipStream_t);                     \
    template hipError_t launch_history<T>(const Geom&, const T*, const T*, const T*,               \
                                          const double*, int, T*, T*, const int*, hipStream_t);    \
    template hipError_t launch_commit_history<T>(const Geom&, const T*, const T*, const double*,   \
                                                 int, T*, const int*, hipStream_t);                \
    template hipError_t launch_pcg_matvec<T>(const Geom&, const uint16_t*, const MatEntry<T>*,     \
                                             const T*, int, double, const T*, T*, double*, int,    \
                                             const PcgDev*, const int*, hipStream_t);              \
    template hipError_t launch_damage_diag<T>(const Geom&, const uint16_t*, const MatEntry<T>*,    \
                                              const T*, int, double, int, T*, double*, int,        \
                                              const int*, hipStream_t);                            \
    template hipError_t launch_pcg_start<T>(const Geom&, const T*, const T*, const T*, T*,         \
                                            double*, int, const int*, hipStream_t);                \
    template hipError_t launch_pcg_update<T>(const Geom&, PcgDev*, T*, T*, const T*, const T*,     \
                                             const T*, double*, int, int, int, hipStream_t);       \
    template hipError_t launch_pcg_matvec_dir<T>(const Geom&, const uint16_t*, const MatEntry<T>*, \
                                                 const T*, int, double, int, const T*, const T*,   \
                                                 const T*, const T*, T*, T*, const double*,        \
                                                 long long, int, const double*, long long, int,    \
                                                 double*, int, PcgDev*, int, hipStream_t);         \
    template hipError_t launch_dissipation<T>(const Geom&, const uint16_t*, const MatEntry<T>*,    \
                                              const T*, double*, int, const int*, hipStream_t);    \
    template hipError_t launch_damage_residual<T>(const Geom&, const uint16_t*,                    \
                                                  const MatEntry<T>*, const T*, const T*,          \
                                                  double*, int, const int*, hipStream_t);          \
    template hipError_t launch_psi_ini<T>(const Geom&, const uint16_t*, const MatEntry<T>*,        \
                                          const T*, T*, const int*, hipStream_t);                  \
    template hipError_t launch_tangent_rhs<T>(const Geom&, const T*, const T*, const T*,           \
                                              const T*, const double*, int, T*, const int*,        \
                                              hipStream_t);                                        \
    template hipError_t launch_dissipation_dir<T>(const Geom&, const uint16_t*,                    \
                                                  const MatEntry<T>*, const T*, const T*,          \
                                                  double*, int, const int*, hipStream_t);          \
    template hipError_t launch_copy<T>(const T*, T*, long long, int, const int*, hipStream_t);     \
    template hipError_t launch_fill<T>(T*, T, long long, int, const int*, hipStream_t);            \
    template hipError_t launch_sub<T>(const T*, const T*, T*, long long, int, const int*,          \
                                      hipStream_t);                                                \
    template hipError_t launch_max_field<T>(const T*, long long, int, double*, int, const int*,    \
                                            hipStream_t);                                          \
    template hipError_t launch_scale_field<T>(T*, const double*, double, long long, int,           \
                                              const int*, hipStream_t);                            \
    template hipError_t launch_diff_norms<T>(const T*, const T*, long long, int, double*, int,     \
                                             const int*, hipStream_t);                             \
    template hipError_t launch_anderson_gram<T>(const Geom&, const T*, long long, const int*,      \
                                                const int*, double*, int, const int*,              \
                                                hipStream_t);                                      \
    template hipError_t launch_anderson_mix<T>(const Geom&, const T*, long long, const int*,       \
                                               const int*, const double*, T*, const int*,          \
                                               hipStream_t);                                       \
    template hipError_t launch_fracture_count<T>(const Geom&, const uint16_t*,                     \
                                                 const MatEntry<T>*, const T*, double, int, int*,  \
                                                 const int*, hipStream_t);

INST(double)
INST(float)

}  // namespace mirve
