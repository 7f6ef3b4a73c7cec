// Pointwise and stencil kernels: unit response, history, the damage
// operator and its Jacobi-preconditioned CG, the AT2 functionals, the
// crack-tip enrichment energy, Anderson mixing, fracture test and the
// finalize kernels of the device-side Krylov scalars.
//
// Damage derivatives are forward differences with periodic wrap; the
// operator L(phi) = -div(G_c l grad phi) (Eq. 10b, 17) is D^T diag(G_c l) D,
// evaluated as a 2d+1 point stencil instead of the paper's FFT form (the two
// are the same linear map).
#include <cfloat>
#include "kernels.h"
#include "reduce.h"

namespace mirve {

constexpr int TPB = 256;

static inline int blocks_for(long long n) {
    long long b = (n + TPB - 1) / TPB;
    return (int)(b < 1 ? 1 : b);
}

template <typename T>
__device__ inline T degr(T phi, T k) {
    const T u = T(1) - phi;
    return u * u + k;
}

struct Nb {
    long long xm, xp, ym, yp, zm, zp;
};

__device__ inline Nb neighbours(const Geom& g, long long idx) {
    const int x = (int)(idx % g.nx);
    const long long t = idx / g.nx;
    const int y = (int)(t % g.ny);
    const int z = (int)(t / g.ny);
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    Nb n;
    n.xm = idx + (x == 0 ? g.nx - 1 : -1);
    n.xp = idx + (x == g.nx - 1 ? -(g.nx - 1) : 1);
    n.ym = idx + (y == 0 ? (g.ny - 1) * sy : -sy);
    n.yp = idx + (y == g.ny - 1 ? -(g.ny - 1) * sy : sy);
    n.zm = idx + (z == 0 ? (g.nz - 1) * sz : -sz);
    n.zp = idx + (z == g.nz - 1 ? -(g.nz - 1) * sz : sz);
    return n;
}

// ---------------------------------------------------------------------------
// finalize kernels (one thread; fixed-order sums)
// ---------------------------------------------------------------------------

// Fixed-order sum of n partials by one block of 256 threads: thread t adds
// entries t, t+256, ... in order, then a fixed tree over the threads.  Every
// thread returns the total.
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

__global__ void k_cg_init(CgDev* cg, const double* prr, int nrr, const double* pb, int nb,
                          double tol, int max_it) {
    const double rr = sum_fixed(prr, nrr);
    const double bn2 = sum_fixed(pb, nb);
    if (threadIdx.x != 0) return;
    cg->rr = rr;
    cg->bn2 = bn2;
    cg->tol2 = tol * tol;
    cg->it = 0;
    cg->first = 1;
    cg->beta = 0.0;
    cg->alpha = 0.0;
    cg->max_it = max_it;
    cg->status = 0;
    cg->done = 0;
    if (!isfinite(rr) || !isfinite(bn2)) { cg->done = 1; cg->status = 2; }
    else if (rr <= cg->tol2 * bn2) { cg->done = 1; cg->status = 1; }
}

__global__ void k_cg_alpha(CgDev* cg, const double* p, int n) {
    if (cg->done) return;
    const double pAp = sum_fixed(p, n);
    if (threadIdx.x != 0) return;
    cg->pAp = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        cg->done = 1;
        cg->status = 2;
        cg->alpha = 0.0;
        return;
    }
    cg->alpha = cg->rr / pAp;
}

__global__ void k_cg_beta(CgDev* cg, const double* p, int n) {
    if (cg->done) return;
    const double rr = sum_fixed(p, n);
    if (threadIdx.x != 0) return;
    cg->beta = rr / cg->rr;
    cg->rr = rr;
    cg->first = 0;
    cg->it += 1;
    if (!isfinite(rr)) { cg->done = 1; cg->status = 2; }
    else if (rr <= cg->tol2 * cg->bn2) { cg->done = 1; cg->status = 1; }
    else if (cg->it >= cg->max_it) { cg->done = 1; cg->status = 3; }
}

hipError_t launch_cg_init(CgDev* cg, const double* prr, int nrr, const double* pb, int nb,
                          double tol, int max_it, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(256), 0, st, cg, prr, nrr, pb, nb, tol, max_it);
    return hipGetLastError();
}
hipError_t launch_cg_alpha(CgDev* cg, const double* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, cg, p, n);
    return hipGetLastError();
}
hipError_t launch_cg_beta(CgDev* cg, const double* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, cg, p, n);
    return hipGetLastError();
}

__global__ void k_sum_partials(const double* p, int stride, int n, int nv, double* out) {
    for (int v = 0; v < nv; ++v) {
        const double s = sum_fixed(p + (long long)v * stride, n);
        if (threadIdx.x == 0) out[v] = s;
    }
}
hipError_t launch_sum_partials(const double* p, int stride, int n, int nv, double* out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, p, stride, n, nv, out);
    return hipGetLastError();
}

__global__ void k_max_partials(const double* p, int n, double* out) {
    if (threadIdx.x != 0) return;
    double m = -DBL_MAX;
    for (int i = 0; i < n; ++i) m = fmax(m, p[i]);
    out[0] = m;
}
hipError_t launch_max_partials(const double* p, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, st, p, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// unit response and history
// ---------------------------------------------------------------------------

struct F6 {
    double v[6];
};

template <typename T, int S>
__global__ void __launch_bounds__(TPB) k_unit_response(Geom g, const uint16_t* mat_id,
                                                       const MatEntry<T>* mat, const T* phi,
                                                       const T* x, F6 f, T* psi1, T* eps1,
                                                       T* sig1, double* partials) {
    double part = 0.0, part2 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const MatEntry<T>& m = mat[mat_id[i]];
        const T gg = degr(phi[i], T(g.k_res));
        T e[S], o[S];
#pragma unroll
        for (int c = 0; c < S; ++c) e[c] = T(f.v[c]) + x[c * g.N + i];
        T psi = T(0);
#pragma unroll
        for (int a = 0; a < S; ++a) {
            T acc = T(0);
#pragma unroll
            for (int b = 0; b < S; ++b) acc += m.C[a * S + b] * e[b];
            o[a] = acc;
            psi += e[a] * acc;
        }
        psi1[i] = T(0.5) * psi * m.drive;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            const T sg = gg * o[c];
            if (eps1) eps1[c * g.N + i] = e[c];
            if (sig1) sig1[c * g.N + i] = sg;
            part += double(sg) * f.v[c];
            part2 += double(sg) * double(sg);
        }
    }
    double pv[2] = {part, part2};
    block_sum_store<2>(pv, partials, kRedBlocks, blockIdx.x);
}

template <typename T>
hipError_t launch_unit_response(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const T* phi, const T* x, const double* f, int split, T* psi1,
                                T* eps1, T* sig1, double* partials, int nblocks, hipStream_t st) {
    (void)split;
    F6 ff;
    for (int c = 0; c < 6; ++c) ff.v[c] = c < g.s ? f[c] : 0.0;
    if (g.s == 3)
        hipLaunchKernelGGL((k_unit_response<T, 3>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id,
                           mat, phi, x, ff, psi1, eps1, sig1, partials);
    else
        hipLaunchKernelGGL((k_unit_response<T, 6>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id,
                           mat, phi, x, ff, psi1, eps1, sig1, partials);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_history(long long N, const T* psi1, const T* psi_ini,
                                                 const T* Hn, T E2, int history, T* H) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T ht = E2 * psi1[i] + psi_ini[i];
    H[i] = history ? (ht > Hn[i] ? ht : Hn[i]) : ht;
}

template <typename T>
hipError_t launch_history(const Geom& g, const T* psi1, const T* psi_ini, const T* Hn, double E,
                          int history, T* H, hipStream_t st) {
    hipLaunchKernelGGL((k_history<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g.N, psi1,
                       psi_ini, Hn, T(E * E), history, H);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_commit_history(const Geom& g, const T* psi1, const T* psi_ini, double E,
                                 int history, T* Hn, hipStream_t st) {
    // in place: H = max(E^2 psi1 + psi_ini, Hn)
    hipLaunchKernelGGL((k_history<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g.N, psi1,
                       psi_ini, (const T*)Hn, T(E * E), history, Hn);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// damage operator and its PCG
// ---------------------------------------------------------------------------

// a(x) and w(x) of the operator a p + D^T (w D p).
template <typename T>
__device__ inline void coeffs(const Geom& g, const MatEntry<T>* mat, const uint16_t* mat_id,
                              const T* H, int mode, T c, long long i, T& a, T& w) {
    if (mode == 0) {
        const T gc = mat[mat_id[i]].Gc;
        a = gc / T(g.ell) + (H ? T(2) * H[i] : T(0));
        w = gc * T(g.ell);
    } else {
        a = T(1);
        w = c;
    }
}

template <typename T>
__device__ inline T wcoef(const MatEntry<T>* mat, const uint16_t* mat_id, int mode, T ell, T c,
                          long long i) {
    return mode == 0 ? mat[mat_id[i]].Gc * ell : c;
}

template <typename T>
__device__ inline T apply_op(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, T c, const T* p, long long i) {
    T a, w;
    coeffs(g, mat, mat_id, H, mode, c, i, a, w);
    const Nb n = neighbours(g, i);
    const T ell = T(g.ell);
    const T ih2 = T(1.0 / (g.h * g.h));
    const T pc = p[i];
    T acc = T(0);
    acc += wcoef(mat, mat_id, mode, ell, c, n.xm) * (pc - p[n.xm]) - w * (p[n.xp] - pc);
    acc += wcoef(mat, mat_id, mode, ell, c, n.ym) * (pc - p[n.ym]) - w * (p[n.yp] - pc);
    if (g.dim == 3)
        acc += wcoef(mat, mat_id, mode, ell, c, n.zm) * (pc - p[n.zm]) - w * (p[n.zp] - pc);
    return a * pc + acc * ih2;
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_matvec(Geom g, const uint16_t* mat_id,
                                                    const MatEntry<T>* mat, const T* H, int mode,
                                                    T c, const T* p, T* q, double* partials,
                                                    const PcgDev* d) {
    if (d && d->done) return;
    double part = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const T v = apply_op(g, mat_id, mat, H, mode, c, p, i);
        q[i] = v;
        part += double(p[i]) * double(v);
    }
    if (partials) {
        double pv[1] = {part};
        block_sum_store<1>(pv, partials, 0, blockIdx.x);
    }
}

template <typename T>
hipError_t launch_pcg_matvec(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, double c, const T* p, T* q, double* partials,
                             int nblocks, const PcgDev* d, hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_matvec<T>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id, mat, H,
                       mode, T(c), p, q, partials, d);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_damage_diag(Geom g, const uint16_t* mat_id,
                                                     const MatEntry<T>* mat, const T* H, int mode,
                                                     T c, T* dinv) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    T a, w;
    coeffs(g, mat, mat_id, H, mode, c, i, a, w);
    const Nb n = neighbours(g, i);
    const T ell = T(g.ell);
    T s = T(2) * w + wcoef(mat, mat_id, mode, ell, c, n.xm) + wcoef(mat, mat_id, mode, ell, c, n.ym);
    if (g.dim == 3) s += w + wcoef(mat, mat_id, mode, ell, c, n.zm);
    dinv[i] = T(1) / (a + s * T(1.0 / (g.h * g.h)));
}

template <typename T>
hipError_t launch_damage_diag(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* H, int mode, double c, T* dinv, hipStream_t st) {
    hipLaunchKernelGGL((k_damage_diag<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g, mat_id,
                       mat, H, mode, T(c), dinv);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_start(long long N, const T* b, const T* Ax,
                                                   const T* dinv, T* r, T* p, double* partials,
                                                   int stride) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const T bi = b[i];
        const T ri = bi - Ax[i];
        const T zi = dinv[i] * ri;
        r[i] = ri;
        p[i] = zi;
        s0 += double(ri) * double(zi);
        s1 += double(ri) * double(ri);
        s2 += double(bi) * double(bi);
    }
    double pv[3] = {s0, s1, s2};
    block_sum_store<3>(pv, partials, stride, blockIdx.x);
}

template <typename T>
hipError_t launch_pcg_start(const Geom& g, const T* b, const T* Ax, const T* dinv, T* r, T* p,
                            double* partials, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_start<T>), dim3(nblocks), dim3(TPB), 0, st, g.N, b, Ax, dinv, r, p,
                       partials, kRedBlocks);
    return hipGetLastError();
}

__global__ void k_pcg_fin_start(PcgDev* d, const double* p, int n, double tol, int max_it) {
    const double rz = sum_fixed(p, n);
    const double rr = sum_fixed(p + kRedBlocks, n);
    const double bn2 = sum_fixed(p + 2 * kRedBlocks, n);
    if (threadIdx.x != 0) return;
    d->rz = rz;
    d->rr = rr;
    d->bn2 = bn2;
    d->tol2 = tol * tol;
    d->it = 0;
    d->max_it = max_it;
    d->status = 0;
    d->done = 0;
    if (!isfinite(d->rr) || !isfinite(d->rz)) { d->done = 1; d->status = 2; }
    else if (d->rr <= d->tol2 * d->bn2) { d->done = 1; d->status = 1; }
}
hipError_t launch_pcg_fin_start(PcgDev* d, const double* p, int n, double tol, int max_it,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_fin_start, dim3(1), dim3(256), 0, st, d, p, n, tol, max_it);
    return hipGetLastError();
}

__global__ void k_pcg_fin_alpha(PcgDev* d, const double* p, int n) {
    if (d->done) return;
    const double pq = sum_fixed(p, n);
    if (threadIdx.x != 0) return;
    d->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) { d->done = 1; d->status = 2; d->alpha = 0.0; return; }
    d->alpha = d->rz / pq;
}
hipError_t launch_pcg_fin_alpha(PcgDev* d, const double* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_fin_alpha, dim3(1), dim3(256), 0, st, d, p, n);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_update(long long N, const PcgDev* d, T* x, T* r,
                                                    const T* p, const T* q, const T* dinv,
                                                    double* partials, int stride) {
    if (d->done) return;
    const T alpha = T(d->alpha);
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        s0 += double(ri) * double(dinv[i] * ri);
        s1 += double(ri) * double(ri);
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, partials, stride, blockIdx.x);
}

template <typename T>
hipError_t launch_pcg_update(const Geom& g, const PcgDev* d, T* x, T* r, const T* p, const T* q,
                             const T* dinv, double* partials, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(nblocks), dim3(TPB), 0, st, g.N, d, x, r, p, q,
                       dinv, partials, kRedBlocks);
    return hipGetLastError();
}

__global__ void k_pcg_fin_beta(PcgDev* d, const double* p, int n) {
    if (d->done) return;
    const double rz = sum_fixed(p, n);
    const double rr = sum_fixed(p + kRedBlocks, n);
    if (threadIdx.x != 0) return;
    d->beta = rz / d->rz;
    d->rz = rz;
    d->rr = rr;
    d->it += 1;
    if (!isfinite(rr) || !isfinite(rz)) { d->done = 1; d->status = 2; }
    else if (rr <= d->tol2 * d->bn2) { d->done = 1; d->status = 1; }
    else if (d->it >= d->max_it) { d->done = 1; d->status = 3; }
}
hipError_t launch_pcg_fin_beta(PcgDev* d, const double* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_fin_beta, dim3(1), dim3(256), 0, st, d, p, n);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pcg_dir(long long N, const PcgDev* d, const T* r,
                                                 const T* dinv, T* p) {
    if (d->done) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    p[i] = dinv[i] * r[i] + T(d->beta) * p[i];
}

template <typename T>
hipError_t launch_pcg_dir(const Geom& g, const PcgDev* d, const T* r, const T* dinv, T* p,
                          hipStream_t st) {
    hipLaunchKernelGGL((k_pcg_dir<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g.N, d, r, dinv,
                       p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AT2 functionals, residual, enrichment energy
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_dissipation(Geom g, const uint16_t* mat_id,
                                                     const MatEntry<T>* mat, const T* phi,
                                                     double* partials, int stride) {
    double sD = 0.0, sG = 0.0;
    const double ell = g.ell, ih = 1.0 / g.h;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double pc = phi[i];
        const double gx = (double(phi[n.xp]) - pc) * ih;
        const double gy = (double(phi[n.yp]) - pc) * ih;
        const double gz = g.dim == 3 ? (double(phi[n.zp]) - pc) * ih : 0.0;
        const double dens = pc * pc / (2.0 * ell) + 0.5 * ell * (gx * gx + gy * gy + gz * gz);
        sD += double(mat[mat_id[i]].Gc) * dens;
        sG += dens;
    }
    double pv[2] = {sD, sG};
    block_sum_store<2>(pv, partials, stride, blockIdx.x);
}

template <typename T>
hipError_t launch_dissipation(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* phi, double* partials, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_dissipation<T>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id, mat, phi,
                       partials, kRedBlocks);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_damage_residual(Geom g, const uint16_t* mat_id,
                                                         const MatEntry<T>* mat, const T* H,
                                                         const T* phi, double* partials,
                                                         int stride) {
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const T v = apply_op(g, mat_id, mat, H, 0, T(0), phi, i);
        const double b = 2.0 * double(H[i]);
        const double res = double(v) - b;
        s0 += res * res;
        s1 += b * b;
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, partials, stride, blockIdx.x);
}

template <typename T>
hipError_t launch_damage_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* H, const T* phi, double* partials, int nblocks,
                                  hipStream_t st) {
    hipLaunchKernelGGL((k_damage_residual<T>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id, mat, H,
                       phi, partials, kRedBlocks);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_psi_ini(Geom g, const uint16_t* mat_id,
                                                 const MatEntry<T>* mat, const T* phi,
                                                 T* psi_ini) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    // gamma'(phi) = Gc phi / l + L phi  (operator with H = 0)
    const T gp = apply_op(g, mat_id, mat, (const T*)nullptr, 0, T(0), phi, i);
    const T v = gp / (T(2) * (T(1) - phi[i]));
    psi_ini[i] = v > T(0) ? v : T(0);
}

template <typename T>
hipError_t launch_psi_ini(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                          const T* phi, T* psi_ini, hipStream_t st) {
    hipLaunchKernelGGL((k_psi_ini<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g, mat_id, mat,
                       phi, psi_ini);
    return hipGetLastError();
}

// Right-hand side of the E-tangent of the damage balance:
// 2 (1 - phi) dH/dE, dH/dE = 2 E psi1 where E^2 psi1 + psi_ini > H^n (or
// everywhere without the history max).
template <typename T>
__global__ void __launch_bounds__(TPB) k_tangent_rhs(long long N, const T* phi, const T* psi1,
                                                     const T* psi_ini, const T* Hn, T E,
                                                     int history, T* out) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T ht = E * E * psi1[i] + psi_ini[i];
    const bool active = history ? (ht > Hn[i]) : true;
    out[i] = active ? T(2) * (T(1) - phi[i]) * T(2) * E * psi1[i] : T(0);
}

template <typename T>
hipError_t launch_tangent_rhs(const Geom& g, const T* phi, const T* psi1, const T* psi_ini,
                              const T* Hn, double E, int history, T* out, hipStream_t st) {
    hipLaunchKernelGGL((k_tangent_rhs<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g.N, phi,
                       psi1, psi_ini, Hn, T(E), history, out);
    return hipGetLastError();
}

// dD(phi)[dphi] = h^d sum Gc (phi dphi / l + l grad phi . grad dphi); partial sums
// without the h^d factor.
template <typename T>
__global__ void __launch_bounds__(TPB) k_dissipation_dir(Geom g, const uint16_t* mat_id,
                                                         const MatEntry<T>* mat, const T* phi,
                                                         const T* dphi, double* partials) {
    double s = 0.0;
    const double ell = g.ell, ih = 1.0 / g.h;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const Nb n = neighbours(g, i);
        const double pc = phi[i], dc = dphi[i];
        double gg = (double(phi[n.xp]) - pc) * (double(dphi[n.xp]) - dc);
        gg += (double(phi[n.yp]) - pc) * (double(dphi[n.yp]) - dc);
        if (g.dim == 3) gg += (double(phi[n.zp]) - pc) * (double(dphi[n.zp]) - dc);
        s += double(mat[mat_id[i]].Gc) * (pc * dc / ell + ell * gg * ih * ih);
    }
    double pv[1] = {s};
    block_sum_store<1>(pv, partials, 0, blockIdx.x);
}

template <typename T>
hipError_t launch_dissipation_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* phi, const T* dphi, double* partials, int nblocks,
                                  hipStream_t st) {
    hipLaunchKernelGGL((k_dissipation_dir<T>), dim3(nblocks), dim3(TPB), 0, st, g, mat_id, mat,
                       phi, dphi, partials);
    return hipGetLastError();
}

// out = a - b
template <typename T>
__global__ void __launch_bounds__(TPB) k_sub(const T* a, const T* b, T* out, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}
template <typename T>
hipError_t launch_sub(const T* a, const T* b, T* out, long long n, hipStream_t st) {
    hipLaunchKernelGGL((k_sub<T>), dim3(blocks_for(n)), dim3(TPB), 0, st, a, b, out, n);
    return hipGetLastError();
}

// b = c * a
template <typename T>
__global__ void __launch_bounds__(TPB) k_scaled(const T* a, T c, T* b, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = c * a[i];
}
template <typename T>
hipError_t launch_scaled(const T* a, double c, T* b, long long n, hipStream_t st) {
    hipLaunchKernelGGL((k_scaled<T>), dim3(blocks_for(n)), dim3(TPB), 0, st, a, T(c), b, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// field utilities
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_copy(const T* s, T* d, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}
template <typename T>
hipError_t launch_copy(const T* s, T* d, long long n, hipStream_t st) {
    hipLaunchKernelGGL((k_copy<T>), dim3(blocks_for(n)), dim3(TPB), 0, st, s, d, n);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_fill(T* d, T v, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}
template <typename T>
hipError_t launch_fill(T* d, T v, long long n, hipStream_t st) {
    hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(n)), dim3(TPB), 0, st, d, v, n);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_max_field(const T* a, long long n, double* partials) {
    double m = -DBL_MAX;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        m = fmax(m, double(a[i]));
    block_max_store(m, partials, blockIdx.x);
}
template <typename T>
hipError_t launch_max_field(const T* a, long long n, double* partials, int nblocks,
                            hipStream_t st) {
    hipLaunchKernelGGL((k_max_field<T>), dim3(nblocks), dim3(TPB), 0, st, a, n, partials);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_scale_field(T* a, const double* den, double c,
                                                     long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) a[i] = T(double(a[i]) * (c / den[0]));
}
template <typename T>
hipError_t launch_scale_field(T* a, const double* den, double c, long long n, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_field<T>), dim3(blocks_for(n)), dim3(TPB), 0, st, a, den, c, n);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_diff_norms(const T* a, const T* b, long long n,
                                                    double* partials, int stride) {
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double d = double(a[i]) - double(b[i]);
        s0 += d * d;
        s1 += double(a[i]) * double(a[i]);
    }
    double pv[2] = {s0, s1};
    block_sum_store<2>(pv, partials, stride, blockIdx.x);
}
template <typename T>
hipError_t launch_diff_norms(const T* a, const T* b, long long n, double* partials, int nblocks,
                             hipStream_t st) {
    hipLaunchKernelGGL((k_diff_norms<T>), dim3(nblocks), dim3(TPB), 0, st, a, b, n, partials,
                       kRedBlocks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Anderson mixing of the stagger iterates
// ---------------------------------------------------------------------------

// Gram data of the residual history F_0..F_m (oldest first):
// values [i*m + j] (i, j < m) = dF_i . dF_j with dF_i = F_{i+1} - F_i,
// values [m*m + i] = dF_i . F_m.
template <typename T, int MM>
__global__ void __launch_bounds__(TPB) k_anderson_gram(long long N, Ptrs<T> F, int m1,
                                                       double* partials, int stride) {
    const int m = m1 - 1;
    double acc[MM * MM + MM];
#pragma unroll
    for (int k = 0; k < MM * MM + MM; ++k) acc[k] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        double f[MM + 1];
#pragma unroll
        for (int k = 0; k <= MM; ++k) f[k] = k < m1 ? double(F.p[k][i]) : 0.0;
        double df[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) df[k] = k < m ? f[k + 1] - f[k] : 0.0;
        const double last = f[m];
#pragma unroll
        for (int a = 0; a < MM; ++a) {
#pragma unroll
            for (int b = 0; b < MM; ++b) acc[a * MM + b] += df[a] * df[b];
            acc[MM * MM + a] += df[a] * last;
        }
    }
    block_sum_store<MM * MM + MM>(acc, partials, stride, blockIdx.x);
}

template <typename T>
hipError_t launch_anderson_gram(const Geom& g, const Ptrs<T>& F, int m1, double* partials,
                                int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_anderson_gram<T, kAndersonMax>), dim3(nblocks), dim3(TPB), 0, st, g.N,
                       F, m1, partials, kRedBlocks);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_anderson_mix(long long N, Ptrs<T> G, int m1, Coef c,
                                                      T* out) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int m = m1 - 1;
    double v = double(G.p[m][i]);
    for (int k = 0; k < m; ++k) v -= c.v[k] * (double(G.p[k + 1][i]) - double(G.p[k][i]));
    out[i] = T(v);
}

template <typename T>
hipError_t launch_anderson_mix(const Geom& g, const Ptrs<T>& G, int m1, const Coef& c, T* out,
                               hipStream_t st) {
    hipLaunchKernelGGL((k_anderson_mix<T>), dim3(blocks_for(g.N)), dim3(TPB), 0, st, g.N, G, m1,
                       c, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fracture test: lines along the load axis without a broken voxel
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(TPB) k_fracture(Geom g, const uint16_t* mat_id,
                                                  const MatEntry<T>* mat, const T* phi, T thr,
                                                  int axis, int* count) {
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
        if (phi[i] >= thr || mat[mat_id[i]].drive == T(0)) broken = true;
    }
    if (!broken) atomicAdd(count, 1);
}

template <typename T>
hipError_t launch_fracture_count(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* phi, double thr, int axis, int* count, hipStream_t st) {
    const long long nlines = g.N / (axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz);
    hipLaunchKernelGGL((k_fracture<T>), dim3(blocks_for(nlines)), dim3(TPB), 0, st, g, mat_id,
                       mat, phi, T(thr), axis, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------

#define INST(T)                                                                                   \
    template hipError_t launch_unit_response<T>(const Geom&, const uint16_t*, const MatEntry<T>*, \
                                                const T*, const T*, const double*, int, T*, T*,   \
                                                T*, double*, int, hipStream_t);                   \
    template hipError_t launch_history<T>(const Geom&, const T*, const T*, const T*, double, int, \
                                          T*, hipStream_t);                                       \
    template hipError_t launch_commit_history<T>(const Geom&, const T*, const T*, double, int,    \
                                                 T*, hipStream_t);                                \
    template hipError_t launch_pcg_matvec<T>(const Geom&, const uint16_t*, const MatEntry<T>*,    \
                                             const T*, int, double, const T*, T*, double*, int,   \
                                             const PcgDev*, hipStream_t);                         \
    template hipError_t launch_damage_diag<T>(const Geom&, const uint16_t*, const MatEntry<T>*,   \
                                              const T*, int, double, T*, hipStream_t);            \
    template hipError_t launch_pcg_start<T>(const Geom&, const T*, const T*, const T*, T*, T*,    \
                                            double*, int, hipStream_t);                           \
    template hipError_t launch_pcg_update<T>(const Geom&, const PcgDev*, T*, T*, const T*,        \
                                             const T*, const T*, double*, int, hipStream_t);      \
    template hipError_t launch_pcg_dir<T>(const Geom&, const PcgDev*, const T*, const T*, T*,     \
                                          hipStream_t);                                           \
    template hipError_t launch_dissipation<T>(const Geom&, const uint16_t*, const MatEntry<T>*,   \
                                              const T*, double*, int, hipStream_t);               \
    template hipError_t launch_damage_residual<T>(const Geom&, const uint16_t*,                   \
                                                  const MatEntry<T>*, const T*, const T*,         \
                                                  double*, int, hipStream_t);                     \
    template hipError_t launch_psi_ini<T>(const Geom&, const uint16_t*, const MatEntry<T>*,       \
                                          const T*, T*, hipStream_t);                             \
    template hipError_t launch_copy<T>(const T*, T*, long long, hipStream_t);                     \
    template hipError_t launch_tangent_rhs<T>(const Geom&, const T*, const T*, const T*,          \
                                              const T*, double, int, T*, hipStream_t);            \
    template hipError_t launch_dissipation_dir<T>(const Geom&, const uint16_t*,                   \
                                                  const MatEntry<T>*, const T*, const T*,         \
                                                  double*, int, hipStream_t);                     \
    template hipError_t launch_scaled<T>(const T*, double, T*, long long, hipStream_t);           \
    template hipError_t launch_sub<T>(const T*, const T*, T*, long long, hipStream_t);            \
    template hipError_t launch_fill<T>(T*, T, long long, hipStream_t);                            \
    template hipError_t launch_max_field<T>(const T*, long long, double*, int, hipStream_t);      \
    template hipError_t launch_scale_field<T>(T*, const double*, double, long long, hipStream_t); \
    template hipError_t launch_diff_norms<T>(const T*, const T*, long long, double*, int,         \
                                             hipStream_t);                                        \
    template hipError_t launch_anderson_gram<T>(const Geom&, const Ptrs<T>&, int, double*, int,   \
                                                hipStream_t);                                     \
    template hipError_t launch_anderson_mix<T>(const Geom&, const Ptrs<T>&, int, const Coef&, T*, \
                                               hipStream_t);                                      \
    template hipError_t launch_fracture_count<T>(const Geom&, const uint16_t*,                    \
                                                 const MatEntry<T>*, const T*, double, int, int*, \
                                                 hipStream_t);

INST(double)
INST(float)

}  // namespace mirve
