// Kernel argument blocks and launchers.
#pragma once
#include "common.h"

namespace mirve {

// Device-resident scalars of one conjugate-gradient solve.  The finalize
// kernels update them so that an iteration needs no host round trip.
struct CgDev {
    double rr;       // r . r of the current residual
    double pAp;      // p . A p
    double alpha, beta;
    double bn2;      // ||b||^2 (stopping reference)
    double tol2;     // tol^2
    int it;          // iterations done
    int done;        // 1 once converged, failed or out of iterations
    int first;       // next direction update is p = r
    int status;      // 0 ok, 1 converged, 2 breakdown / non-finite, 3 max iterations
    int max_it;
    int pad;
};

enum { XF_GREEN = 0, XF_CG = 1 };
enum { AX_FWD = 0, AX_INV = 1, AX_FWD_P_INV = 2 };
enum { XI_STORE = 0, XI_CG = 1 };

template <typename T>
struct XfwdArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    const uint16_t* mat_id;
    const MatEntry<T>* mat;
    const T* phi;
    const T* eps;        // XF_GREEN: strain field (s*N) or null
    T fcoef;             // XF_GREEN: + fcoef * f
    T f[6];
    const T* r;          // XF_CG
    T* p;                // XF_CG (updated in place)
    const CgDev* cg;     // XF_CG
    cplx<T>* spec;
    double* partials;
    int rows_per_block;
};

template <typename T>
struct AxisArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    cplx<T>* spec;
    const CgDev* cg;     // skip when cg && cg->done
    int axis;            // 1 = y, 2 = z
    int tx;              // kx columns per block
};

template <typename T>
struct XinvArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    const cplx<T>* spec;
    T scale;             // multiplies the (normalised) inverse
    T* out;              // XI_STORE (may be null: norm only)
    T* x;                // XI_CG
    const T* p;          // XI_CG
    T* r;                // XI_CG
    const CgDev* cg;
    double* partials;
    int rows_per_block;
};

template <typename T>
hipError_t launch_xfwd(const XfwdArgs<T>& a, int mode, int maxb, int nblocks, size_t lds,
                       hipStream_t st);
template <typename T>
hipError_t launch_axis(const AxisArgs<T>& a, int mode, int maxb, dim3 grid, size_t lds,
                       hipStream_t st);
template <typename T>
hipError_t launch_xinv(const XinvArgs<T>& a, int mode, int maxb, int nblocks, size_t lds,
                       hipStream_t st);

// ---------------------------------------------------------------------------
// pointwise / stencil kernels (pointwise.hip)
// ---------------------------------------------------------------------------

// Finalize kernels for the mechanics CG.
hipError_t launch_cg_init(CgDev* cg, const double* partials_rr, int nrr, const double* partials_b,
                          int nb, double tol, int max_it, hipStream_t st);
hipError_t launch_cg_alpha(CgDev* cg, const double* partials, int n, hipStream_t st);
hipError_t launch_cg_beta(CgDev* cg, const double* partials, int n, hipStream_t st);

// Sum (fixed order) nv groups of n partials: out[v] = sum_b partials[v*stride + b].
hipError_t launch_sum_partials(const double* partials, int stride, int n, int nv, double* out,
                               hipStream_t st);
hipError_t launch_max_partials(const double* partials, int n, double* out, hipStream_t st);

// Unit response: eps1 = f + x, sigma1 = g C eps1, psi1 (0 on notch voxels),
// partial sums of sigma1:f (slot 0) and sigma1:sigma1 (slot 1, stride
// kRedBlocks).  Also writes eps1/sig1 if non-null.
template <typename T>
hipError_t launch_unit_response(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const T* phi, const T* x, const double* f, int split, T* psi1,
                                T* eps1, T* sig1, double* partials, int nblocks, hipStream_t st);

// History at load E: H = max(E^2 psi1 + psi_ini, Hn) (or without max),
// optionally its E-derivative mask.
template <typename T>
hipError_t launch_history(const Geom& g, const T* psi1, const T* psi_ini, const T* Hn, double E,
                          int history, T* H, hipStream_t st);

// Damage operator q = a(x) p + D^T (w(x) D p) with a = Gc/l + 2H, w = Gc l
// (coefficient mode 0; H may be null) or a = 1, w = c (mode 1, the
// enrichment smoothing).  See launch_pcg_matvec.

// Jacobi diagonal of the damage operator.
template <typename T>
hipError_t launch_damage_diag(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* H, int mode, double c, T* dinv, hipStream_t st);

// Jacobi-preconditioned CG of the damage system; scalars live on the device.
struct PcgDev {
    double rz, pq, alpha, beta, rr, bn2, tol2;
    int it, done, status, max_it;
};
// r = b - Ax, p = z = dinv r; partials: r.z, r.r, b.b
template <typename T>
hipError_t launch_pcg_start(const Geom& g, const T* b, const T* Ax, const T* dinv, T* r, T* p,
                            double* partials, int nblocks, hipStream_t st);
hipError_t launch_pcg_fin_start(PcgDev* d, const double* partials, int n, double tol, int max_it,
                                hipStream_t st);
// q = A p with p.q partials, skipped once done
template <typename T>
hipError_t launch_pcg_matvec(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, double c, const T* p, T* q, double* partials,
                             int nblocks, const PcgDev* d, hipStream_t st);
hipError_t launch_pcg_fin_alpha(PcgDev* d, const double* partials, int n, hipStream_t st);
// x += alpha p; r -= alpha q; partials r.(dinv r), r.r
template <typename T>
hipError_t launch_pcg_update(const Geom& g, const PcgDev* d, T* x, T* r, const T* p, const T* q,
                             const T* dinv, double* partials, int nblocks, hipStream_t st);
hipError_t launch_pcg_fin_beta(PcgDev* d, const double* partials, int n, hipStream_t st);
// p = dinv r + beta p
template <typename T>
hipError_t launch_pcg_dir(const Geom& g, const PcgDev* d, const T* r, const T* dinv, T* p,
                          hipStream_t st);

// Dissipation D(phi) and Gamma(phi) partial sums (Eq. 3, 4).
template <typename T>
hipError_t launch_dissipation(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* phi, double* partials, int nblocks, hipStream_t st);

// Damage residual norm partials: ||(Gc/l + 2H) phi + L phi - 2H||^2 and ||2H||^2.
template <typename T>
hipError_t launch_damage_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* H, const T* phi, double* partials, int nblocks,
                                  hipStream_t st);

// Field utilities.
template <typename T>
hipError_t launch_copy(const T* src, T* dst, long long n, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* dst, T v, long long n, hipStream_t st);
template <typename T>
hipError_t launch_max_field(const T* a, long long n, double* partials, int nblocks, hipStream_t st);
template <typename T>
hipError_t launch_scale_field(T* a, const double* num, double c, long long n, hipStream_t st);
// psi_ini = max(0, gamma'(phi) / (2 (1 - phi))) (Eq. 37a)
template <typename T>
hipError_t launch_psi_ini(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                          const T* phi, T* psi_ini, hipStream_t st);
// Anderson mixing of the stagger iterates (depth <= kAndersonMax).
constexpr int kAndersonMax = 5;
template <typename T>
struct Ptrs {
    const T* p[kAndersonMax + 1];
};
struct Coef {
    double v[kAndersonMax];
};
// Gram data of residual history F_0..F_m (oldest first, m1 = m + 1 <= kAndersonMax + 1):
// value a*kAndersonMax + b = dF_a . dF_b, value kAndersonMax^2 + a = dF_a . F_m,
// dF_a = F_{a+1} - F_a.  Partials are strided by kRedBlocks.
template <typename T>
hipError_t launch_anderson_gram(const Geom& g, const Ptrs<T>& F, int m1, double* partials,
                                int nblocks, hipStream_t st);
// out = G_m - sum_a gamma_a (G_{a+1} - G_a)
template <typename T>
hipError_t launch_anderson_mix(const Geom& g, const Ptrs<T>& G, int m1, const Coef& c, T* out,
                               hipStream_t st);
// ||a - b||^2 and ||a||^2 partials
template <typename T>
hipError_t launch_diff_norms(const T* a, const T* b, long long n, double* partials, int nblocks,
                             hipStream_t st);
// number of lines along the load axis without a broken voxel
template <typename T>
hipError_t launch_fracture_count(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* phi, double thr, int axis, int* count, hipStream_t st);
// 2 (1 - phi) dH/dE (right-hand side of the E-tangent of the damage balance)
template <typename T>
hipError_t launch_tangent_rhs(const Geom& g, const T* phi, const T* psi1, const T* psi_ini,
                              const T* Hn, double E, int history, T* out, hipStream_t st);
// partials of sum Gc (phi dphi / l + l grad phi . grad dphi)
template <typename T>
hipError_t launch_dissipation_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* phi, const T* dphi, double* partials, int nblocks,
                                  hipStream_t st);
// out = a - b
template <typename T>
hipError_t launch_sub(const T* a, const T* b, T* out, long long n, hipStream_t st);
// b = c a
template <typename T>
hipError_t launch_scaled(const T* a, double c, T* b, long long n, hipStream_t st);
// Commit history: Hn = max(E^2 psi1 + psi_ini, Hn)  (or no max)
template <typename T>
hipError_t launch_commit_history(const Geom& g, const T* psi1, const T* psi_ini, double E,
                                 int history, T* Hn, hipStream_t st);

}  // namespace mirve
