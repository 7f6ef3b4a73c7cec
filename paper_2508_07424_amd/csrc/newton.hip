// Kernels of the monolithic Newton-Raphson step (Sec. 4.1, Eq. 22-31):
// the pointwise parts of the residual R = (R1, R2, R3) of Eq. 24 and of the
// Jacobian J = (J1, J2, J3) of Eq. 25, and the vector kernels of the
// restarted GMRES that solves each Newton system J dq = -R.
//
// One RVE per launch, FP64 only.  Field pointers are already offset to that
// RVE.  A Newton vector q = (x, phi, E) is stored flat: the s strain
// components of the fluctuation x (component-major, s * N values), then
// phi (N values), then E (one value), n = (s + 1) N + 1 in all.
//
// Reductions write per-block partial sums that a second kernel adds in a
// fixed order, so every result is bitwise reproducible for a fixed launch
// shape.
#include "newton.h"
#include "reduce.h"

namespace mirve {

namespace {

constexpr int TPB = 256;

int grid_for(long long n, int cap) {
    long long b = (n + TPB - 1) / TPB;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

__device__ inline double degr64(double phi, double k) {
    const double u = 1.0 - phi;
    return u * u + k;
}

// strain e = x + E f at voxel i, undegraded stress o = C : e, energy
// psi0 = 1/2 e : C : e (0 on notch voxels)
template <int S>
__device__ inline double point_state(const NrArgs& a, long long i, double (&e)[S], double (&o)[S],
                                     const MatEntry<double>*& m) {
    m = &a.mat[a.mat_id[i]];
#pragma unroll
    for (int c = 0; c < S; ++c) e[c] = a.x[c * a.g.N + i] + a.E * a.f.v[c];
    double psi = 0.0;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < S; ++c) acc += m->C[r * S + c] * e[c];
        o[r] = acc;
        psi += e[r] * acc;
    }
    return 0.5 * psi * m->drive;
}

// H = max(psi0 + psi_ini, H^n) (Eq. 38; without the history, psi0 + psi_ini)
template <int S>
__global__ void __launch_bounds__(TPB) k_nr_history(NrArgs a, double* H) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.g.N;
         i += (long long)gridDim.x * blockDim.x) {
        double e[S], o[S];
        const MatEntry<double>* m;
        const double ht = point_state<S>(a, i, e, o, m) + a.psi_ini[i];
        H[i] = a.history ? fmax(ht, a.Hn[i]) : ht;
    }
}

// Pointwise part of J applied to dq = (dx, dphi, dE):
//   w  = (g de + g' dphi e) / g(0), de = dx + dE f, so that the Green
//        operator of the law at phi = 0 gives J1 = Gamma[g C de + g' sigma0 dphi];
//   t2 = g' dH with dH = sigma0 : de where the history follows psi0
//        (psi0 + psi_ini >= H^n, psi0 > 0, not a notch voxel), else 0;
//   dphi copied out for the stencil kernels.
template <int S>
__global__ void __launch_bounds__(TPB) k_nr_jac_point(NrArgs a, const double* dq, double inv_g0,
                                                     double* w, double* dphi_out, double* t2) {
    const long long N = a.g.N;
    const double dE = dq[(long long)S * N + N];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        double e[S], o[S], de[S];
        const MatEntry<double>* m;
        const double psi0 = point_state<S>(a, i, e, o, m);
        const double ph = a.phi[i];
        const double dph = dq[(long long)S * N + i];
        const double gg = degr64(ph, a.g.k_res);
        const double gp = -2.0 * (1.0 - ph);
        double dH = 0.0;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            de[c] = dq[c * N + i] + dE * a.f.v[c];
            w[c * N + i] = (gg * de[c] + gp * dph * e[c]) * inv_g0;
            dH += o[c] * de[c];
        }
        const double ht = psi0 + a.psi_ini[i];
        const bool act = (!a.history || ht >= a.Hn[i]) && m->drive != 0.0 && psi0 > 0.0;
        t2[i] = act ? gp * dH : 0.0;
        dphi_out[i] = dph;
    }
}

// out = (cx xs, ca a + cb b, escale * esrc[0] + eadd); b and esrc may be null
__global__ void __launch_bounds__(TPB) k_nr_pack(long long sN, long long N, double* out,
                                                const double* xs, double cx, const double* a,
                                                double ca, const double* b, double cb,
                                                const double* esrc, double escale, double eadd) {
    const long long n = sN + N + 1;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double v;
        if (i < sN) {
            v = cx * xs[i];
        } else if (i < sN + N) {
            const long long j = i - sN;
            v = ca * a[j] + (b ? cb * b[j] : 0.0);
        } else {
            v = (esrc ? escale * esrc[0] : 0.0) + eadd;
        }
        out[i] = v;
    }
}

// partials[j * nblk + block] = block's share of V_j . w, j < k (grid: nblk x k)
__global__ void __launch_bounds__(TPB) k_mdot(const double* V, long long ldv, const double* w,
                                             long long n, double* partials) {
    const int j = blockIdx.y;
    const double* v = V + (long long)j * ldv;
    double s = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        s += v[i] * w[i];
    double pv[1] = {s};
    block_sum_store<1>(pv, partials + (long long)j * gridDim.x, 1, blockIdx.x);
}

// out[j] = V_j . w by one block per j (short vectors: no second launch)
__global__ void __launch_bounds__(TPB) k_mdot1(const double* V, long long ldv, const double* w,
                                              long long n, double* out) {
    const double* v = V + (long long)blockIdx.x * ldv;
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) s += v[i] * w[i];
    double pv[1] = {s};
    block_sum_store<1>(pv, out, 1, blockIdx.x);
}

// out[j] = sum of partials[j * nblk + 0 .. nblk) in a fixed order (one block per j)
__global__ void __launch_bounds__(TPB) k_mdot_fin(const double* partials, int nblk, double* out) {
    const int j = blockIdx.x;
    double s[1];
    block_sum_all<1>(partials + (long long)j * nblk, 0, nblk, s);
    if (threadIdx.x == 0) out[j] = s[0];
}

// w += alpha * sum_{j < k} c[j] V_j.  A block covers 32 consecutive entries
// with 8 groups of 32 lanes; group q adds the vectors j = q, q + 8, ...;
// the 8 group sums are then added in order.
constexpr int kAxpyLanes = 32, kAxpyGroups = TPB / kAxpyLanes;

__global__ void __launch_bounds__(TPB) k_maxpy(const double* V, long long ldv, int k, const double* c,
                                              double alpha, double* w, long long n) {
    __shared__ double part[kAxpyGroups][kAxpyLanes];
    const int lane = threadIdx.x % kAxpyLanes, q = threadIdx.x / kAxpyLanes;
    for (long long base = (long long)blockIdx.x * kAxpyLanes; base < n;
         base += (long long)gridDim.x * kAxpyLanes) {
        const long long i = base + lane;
        double acc = 0.0;
        if (i < n)
            for (int j = q; j < k; j += kAxpyGroups) acc += c[j] * V[(long long)j * ldv + i];
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0 && i < n) {
            double sum = 0.0;
            for (int r = 0; r < kAxpyGroups; ++r) sum += part[r][lane];
            w[i] += alpha * sum;
        }
        __syncthreads();
    }
}

// Givens rotations of the Arnoldi process.  gv = beta e_1.
__global__ void k_gmres_start(double* gv, int m, const double* nrm2) {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) gv[i] = i == 0 ? sqrt(fmax(nrm2[0], 0.0)) : 0.0;
}

constexpr int kMaxRestart = 1000;

// Column j of the Hessenberg matrix (first and second Gram-Schmidt passes,
// the new vector's norm^2 at hB[j + 1]) rotated by the previous rotations;
// a new rotation zeroes its subdiagonal.  est[j] = |residual| after column
// j, NaN at a breakdown.  The block stages the column and the rotations in
// LDS; one thread applies the rotation chain.
__global__ void __launch_bounds__(TPB) k_gmres_col(int j, int ldr, const double* hA, const double* hB,
                                                  double* R, double* cs, double* sn, double* gv,
                                                  double* est) {
    __shared__ double c_col[kMaxRestart + 1], c_cs[kMaxRestart], c_sn[kMaxRestart];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        c_col[i] = hA[i] + hB[i];
        if (i < j) { c_cs[i] = cs[i]; c_sn[i] = sn[i]; }
    }
    __syncthreads();
    double* col = R + (long long)j * ldr;
    if (threadIdx.x == 0) {
        const double hn2 = hB[j + 1];
        double lo = hn2 > 0.0 ? sqrt(hn2) : 0.0;
        // rotation i mixes entries i and i + 1; entry i + 1 is carried to the next
        double carry = c_col[0];
        for (int i = 0; i < j; ++i) {
            const double nxt = c_col[i + 1];
            c_col[i] = c_cs[i] * carry + c_sn[i] * nxt;
            carry = -c_sn[i] * carry + c_cs[i] * nxt;
        }
        const double rr = hypot(carry, lo);
        if (!(rr > 0.0) || !isfinite(rr)) {
            est[j] = __builtin_nan("");
            c_col[j] = carry;
        } else {
            const double cj = carry / rr, sj = lo / rr;
            cs[j] = cj;
            sn[j] = sj;
            c_col[j] = rr;
            const double g = gv[j];
            gv[j + 1] = -sj * g;
            gv[j] = cj * g;
            est[j] = fabs(sj * g);
        }
        col[j + 1] = 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = c_col[i];
}

// y = R^-1 gv over the first k columns: column-oriented back substitution,
// the right-hand side in LDS, one barrier per column
__global__ void __launch_bounds__(TPB) k_gmres_solve(int k, int ldr, const double* R, const double* gv,
                                                    double* y) {
    __shared__ double rhs[kMaxRestart];
    __shared__ double yi;
    for (int i = threadIdx.x; i < k; i += blockDim.x) rhs[i] = gv[i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double* ci = R + (long long)i * ldr;
        if (threadIdx.x == 0) {
            yi = rhs[i] / ci[i];
            y[i] = yi;
        }
        __syncthreads();
        const double v = yi;
        for (int l = threadIdx.x; l < i; l += blockDim.x) rhs[l] -= ci[l] * v;
        __syncthreads();
    }
}

// w /= sqrt(nrm2[0]) (left as it is when nrm2 is not positive)
__global__ void __launch_bounds__(TPB) k_unit_scale(double* w, long long n, const double* nrm2) {
    const double s2 = nrm2[0];
    if (!(s2 > 0.0)) return;
    const double inv = 1.0 / sqrt(s2);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        w[i] *= inv;
}

// y = a x + b y (y = a x when b == 0, whatever y held)
__global__ void __launch_bounds__(TPB) k_axpby(long long n, double a, const double* x, double b,
                                              double* y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// Newton update x += alpha dx, phi += alpha dphi, with the partial sums of
// |dx + dE f|^2, |x_new + E_new f|^2, |dphi|^2 and |phi_new|^2 (Eq. 30)
template <int S>
__global__ void __launch_bounds__(TPB) k_nr_update(long long N, const double* dq, double alpha,
                                                  F6 f, double E_new, double* x, double* phi,
                                                  double* partials) {
    const double dE = dq[(long long)S * N + N];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < S; ++c) {
            const double dx = dq[c * N + i];
            const double de = dx + dE * f.v[c];
            const double xn = x[c * N + i] + alpha * dx;
            x[c * N + i] = xn;
            const double e = xn + E_new * f.v[c];
            s[0] += de * de;
            s[1] += e * e;
        }
        const double dp = dq[(long long)S * N + i];
        const double pn = phi[i] + alpha * dp;
        phi[i] = pn;
        s[2] += dp * dp;
        s[3] += pn * pn;
    }
    block_sum_store<4>(s, partials, gridDim.x, blockIdx.x);
}

}  // namespace

hipError_t launch_nr_history(const NrArgs& a, double* H, hipStream_t st) {
    const dim3 grid(grid_for(a.g.N, 1024));
    if (a.g.s == 3) hipLaunchKernelGGL((k_nr_history<3>), grid, dim3(TPB), 0, st, a, H);
    else hipLaunchKernelGGL((k_nr_history<6>), grid, dim3(TPB), 0, st, a, H);
    return hipGetLastError();
}

hipError_t launch_nr_jac_point(const NrArgs& a, const double* dq, double inv_g0, double* w,
                               double* dphi_out, double* t2, hipStream_t st) {
    const dim3 grid(grid_for(a.g.N, 1024));
    if (a.g.s == 3)
        hipLaunchKernelGGL((k_nr_jac_point<3>), grid, dim3(TPB), 0, st, a, dq, inv_g0, w, dphi_out, t2);
    else
        hipLaunchKernelGGL((k_nr_jac_point<6>), grid, dim3(TPB), 0, st, a, dq, inv_g0, w, dphi_out, t2);
    return hipGetLastError();
}

hipError_t launch_nr_pack(long long sN, long long N, double* out, const double* xs, double cx,
                          const double* a, double ca, const double* b, double cb,
                          const double* esrc, double escale, double eadd, hipStream_t st) {
    hipLaunchKernelGGL(k_nr_pack, dim3(grid_for(sN + N + 1, 2048)), dim3(TPB), 0, st, sN, N, out,
                       xs, cx, a, ca, b, cb, esrc, escale, eadd);
    return hipGetLastError();
}

int nr_dot_blocks(long long n) { return grid_for(n, 64); }

// vectors up to this length take one block per dot product
constexpr long long kMdotOneBlock = 1 << 16;

hipError_t launch_mdot(const double* V, long long ldv, int k, const double* w, long long n,
                       double* partials, double* out, hipStream_t st) {
    if (n <= kMdotOneBlock) {
        hipLaunchKernelGGL(k_mdot1, dim3(k), dim3(TPB), 0, st, V, ldv, w, n, out);
        return hipGetLastError();
    }
    const int nblk = nr_dot_blocks(n);
    hipLaunchKernelGGL(k_mdot, dim3(nblk, k), dim3(TPB), 0, st, V, ldv, w, n, partials);
    hipLaunchKernelGGL(k_mdot_fin, dim3(k), dim3(TPB), 0, st, partials, nblk, out);
    return hipGetLastError();
}

hipError_t launch_maxpy(const double* V, long long ldv, int k, const double* c, double alpha,
                        double* w, long long n, hipStream_t st) {
    long long nb = (n + kAxpyLanes - 1) / kAxpyLanes;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_maxpy, dim3((unsigned)nb), dim3(TPB), 0, st, V, ldv, k, c, alpha, w, n);
    return hipGetLastError();
}

hipError_t launch_gmres_start(double* gv, int m, const double* nrm2, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(TPB), 0, st, gv, m, nrm2);
    return hipGetLastError();
}

hipError_t launch_gmres_col(int j, int ldr, const double* hA, const double* hB, double* R, double* cs,
                            double* sn, double* gv, double* est, hipStream_t st) {
    if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gmres_col, dim3(1), dim3(TPB), 0, st, j, ldr, hA, hB, R, cs, sn, gv, est);
    return hipGetLastError();
}

hipError_t launch_gmres_solve(int k, int ldr, const double* R, const double* gv, double* y,
                              hipStream_t st) {
    if (k < 0 || k > kMaxRestart) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(TPB), 0, st, k, ldr, R, gv, y);
    return hipGetLastError();
}

hipError_t launch_unit_scale(double* w, long long n, const double* nrm2, hipStream_t st) {
    hipLaunchKernelGGL(k_unit_scale, dim3(grid_for(n, 2048)), dim3(TPB), 0, st, w, n, nrm2);
    return hipGetLastError();
}

hipError_t launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 2048)), dim3(TPB), 0, st, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t launch_nr_update(int s, long long N, const double* dq, double alpha, const F6& f,
                            double E_new, double* x, double* phi, double* partials, double* out,
                            hipStream_t st) {
    const int nblk = nr_dot_blocks(N);
    if (s == 3)
        hipLaunchKernelGGL((k_nr_update<3>), dim3(nblk), dim3(TPB), 0, st, N, dq, alpha, f, E_new,
                           x, phi, partials);
    else
        hipLaunchKernelGGL((k_nr_update<6>), dim3(nblk), dim3(TPB), 0, st, N, dq, alpha, f, E_new,
                           x, phi, partials);
    hipLaunchKernelGGL(k_mdot_fin, dim3(4), dim3(TPB), 0, st, partials, nblk, out);
    return hipGetLastError();
}

}  // namespace mirve
