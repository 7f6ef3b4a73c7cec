// Kernel argument blocks and launchers.
//
// Every kernel works on a batch of B RVEs of the same grid.  Fields of RVE b
// start at b * (field size); the launch grid carries the RVE index in its
// last dimension.  Per-RVE scalars (Krylov state, loads, mixing weights)
// live in device arrays indexed by b.  An optional mask active[b] lets a
// launch skip RVEs that have finished a phase.
#pragma once
#include "common.h"

namespace mirve {

constexpr int kMaxVals = 32;       // reduction values per RVE (partials / sums slots)
constexpr int kAndersonMax = 5;    // Anderson depth limit
constexpr int kHist = kAndersonMax + 1;

// Device-resident scalars of one conjugate-gradient solve (one per RVE).
struct CgDev {
    double rr;       // r . r of the current residual
    double pAp;      // p . A p
    double alpha, beta;
    double bn2;      // ||b||^2 (stopping reference)
    double tol2;     // tol^2
    int it;          // iterations done
    int done;        // 1 once converged, failed or out of iterations (or inactive)
    int first;       // next direction update is p = r
    int status;      // 0 running, 1 converged, 2 breakdown / non-finite, 3 max iterations
    int max_it;
    int pad;
};

// Jacobi-preconditioned CG of the damage system (one per RVE).
struct PcgDev {
    double rz, pq, alpha, beta, rr, bn2, tol2;
    int it, done, status, max_it;
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
    const T* eps;        // XF_GREEN: strain field (s*N per RVE) or null
    T fcoef;             // XF_GREEN: + fcoef * f
    T f[6];
    const T* r;          // XF_CG
    T* p;                // XF_CG (updated in place)
    const CgDev* cg;     // XF_CG: per-RVE state; XF_GREEN: null
    const int* active;   // XF_GREEN: optional per-RVE mask
    cplx<T>* spec;
    double* partials;    // [B][nblocks]
    int rows_per_block;
    int nblocks;
    int threads;         // block size (multiple of 64, <= 256)
};

template <typename T>
struct AxisArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    cplx<T>* spec;
    const CgDev* cg;     // skip RVE b when cg && cg[b].done
    const int* active;   // or when active && !active[b]
    int contiguous;      // 1: y lines (stride 1); 0: z lines (stride n_y)
    int lines;           // lines per block (y pass) / y columns per block (z pass)
    int threads;         // block size (multiple of 64, <= 256)
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
    const int* active;
    double* partials;    // [B][nblocks]
    int rows_per_block;
    int nblocks;
    int threads;         // block size (multiple of 64, <= 256)
};

template <typename T>
hipError_t launch_xfwd(const XfwdArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_axis(const AxisArgs<T>& a, int mode, int maxb, dim3 grid, size_t lds,
                       hipStream_t st);
template <typename T>
hipError_t launch_xinv(const XinvArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st);

// ---------------------------------------------------------------------------
// finalize kernels (one block per RVE, fixed-order sums)
// ---------------------------------------------------------------------------

// CG partials are [B][n] (one per block of the pass that made them).
hipError_t launch_cg_init(CgDev* cg, const double* prr, const double* pb, int n, int B,
                          double tol, int max_it, const int* active, hipStream_t st);
hipError_t launch_cg_alpha(CgDev* cg, const double* partials, int n, int B, hipStream_t st);
hipError_t launch_cg_beta(CgDev* cg, const double* partials, int n, int B, hipStream_t st);
// sums[b*kMaxVals + v] = sum_k partials[(b*kMaxVals + v)*kRedBlocks + k], v < nv
hipError_t launch_sum_partials(const double* partials, int n, int nv, int B, double* sums,
                               const int* active, hipStream_t st);
// sums[b*kMaxVals + slot] = sum_k p[b*n + k]  (pass partials)
hipError_t launch_sum_rows(const double* p, int n, int B, double* sums, int slot, hipStream_t st);
// sums[b*kMaxVals] = max_k partials[(b*kMaxVals)*kRedBlocks + k]
hipError_t launch_max_partials(const double* partials, int n, int B, double* sums,
                               const int* active, hipStream_t st);

// Damage PCG partials use the kMaxVals layout above.
hipError_t launch_pcg_fin_start(PcgDev* d, const double* partials, int n, int B, double tol,
                                int max_it, const int* active, hipStream_t st);
hipError_t launch_pcg_fin_alpha(PcgDev* d, const double* partials, int n, int B, hipStream_t st);
hipError_t launch_pcg_fin_beta(PcgDev* d, const double* partials, int n, int B, hipStream_t st);

// ---------------------------------------------------------------------------
// pointwise / stencil kernels; `nred` blocks per RVE for reductions
// ---------------------------------------------------------------------------

struct F6 {
    double v[6];
};

// eps1 = f + x, sigma1 = g C eps1, psi1 (0 on notch voxels); partial sums of
// sigma1:f (value 0) and sigma1:sigma1 (value 1); eps1 / sig1 written if non-null.
template <typename T>
hipError_t launch_unit_response(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const T* phi, const T* x, const F6& f, T* psi1, T* eps1, T* sig1,
                                double* partials, int nred, const int* active, hipStream_t st);

// H = max(E_b^2 psi1 + psi_ini, Hn) (history) or E_b^2 psi1 + psi_ini; rhs = 2H.
template <typename T>
hipError_t launch_history(const Geom& g, const T* psi1, const T* psi_ini, const T* Hn,
                          const double* E, int history, T* H, T* rhs, const int* active,
                          hipStream_t st);

// Damage operator q = a(x) p + D^T (w(x) D p): mode 0 a = Gc/l + 2H (H may be
// null), w = Gc l; mode 1 a = 1, w = c (the enrichment smoothing).
template <typename T>
hipError_t launch_damage_diag(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* H, int mode, double c, T* dinv, const int* active,
                              hipStream_t st);
template <typename T>
hipError_t launch_pcg_matvec(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, double c, const T* p, T* q, double* partials,
                             int nred, const PcgDev* d, const int* active, hipStream_t st);
// r = b - Ax, p = dinv r; partials r.z, r.r, b.b
template <typename T>
hipError_t launch_pcg_start(const Geom& g, const T* b, const T* Ax, const T* dinv, T* r, T* p,
                            double* partials, int nred, const int* active, hipStream_t st);
// One PCG iteration: (1) direction and operator: p_new = dinv r + beta p_old
// evaluated at the voxel and its stencil neighbours, q = A p_new, partials
// p.q; (2) alpha; (3) update: x += alpha p, r -= alpha q, partials r.z, r.r;
// (4) beta and convergence.
template <typename T>
hipError_t launch_pcg_matvec_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* H, int mode, double c, const T* r, const T* dinv,
                                 const T* p_old, T* p_new, T* q, double* partials, int nred,
                                 const PcgDev* d, hipStream_t st);
template <typename T>
hipError_t launch_pcg_update(const Geom& g, const PcgDev* d, T* x, T* r, const T* p, const T* q,
                             const T* dinv, double* partials, int nred, hipStream_t st);

// D(phi) (value 0) and Gamma(phi) (value 1) partials without the h^d factor.
template <typename T>
hipError_t launch_dissipation(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* phi, double* partials, int nred, const int* active,
                              hipStream_t st);
// ||(Gc/l + 2H) phi + L phi - 2H||^2 (value 0) and ||2H||^2 (value 1)
template <typename T>
hipError_t launch_damage_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* H, const T* phi, double* partials, int nred,
                                  const int* active, hipStream_t st);
// psi_ini = max(0, gamma'(phi) / (2 (1 - phi))) (Eq. 37a)
template <typename T>
hipError_t launch_psi_ini(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                          const T* phi, T* psi_ini, const int* active, hipStream_t st);
// 2 (1 - phi) dH/dE with dH/dE = 2 E psi1 where E^2 psi1 + psi_ini > Hn (or everywhere)
template <typename T>
hipError_t launch_tangent_rhs(const Geom& g, const T* phi, const T* psi1, const T* psi_ini,
                              const T* Hn, const double* E, int history, T* out,
                              const int* active, hipStream_t st);
// sum Gc (phi dphi / l + l grad phi . grad dphi) partials (value 0)
template <typename T>
hipError_t launch_dissipation_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                  const T* phi, const T* dphi, double* partials, int nred,
                                  const int* active, hipStream_t st);

// Field utilities over n elements per RVE (stride n).
template <typename T>
hipError_t launch_copy(const T* src, T* dst, long long n, int B, const int* active, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* dst, T v, long long n, int B, const int* active, hipStream_t st);
template <typename T>
hipError_t launch_sub(const T* a, const T* b, T* out, long long n, int B, const int* active,
                      hipStream_t st);
// max over the field (value 0) per RVE
template <typename T>
hipError_t launch_max_field(const T* a, long long n, int B, double* partials, int nred,
                            const int* active, hipStream_t st);
// a *= c / den[b * kMaxVals]
template <typename T>
hipError_t launch_scale_field(T* a, const double* den, double c, long long n, int B,
                              const int* active, hipStream_t st);
// ||a - b||^2 (value 0) and ||a||^2 (value 1)
template <typename T>
hipError_t launch_diff_norms(const T* a, const T* b, long long n, int B, double* partials,
                             int nred, const int* active, hipStream_t st);

// Anderson mixing.  History slot k of every RVE is a batched field at
// base + k * slot_stride; order[b * kHist + i] (i < m1[b]) lists RVE b's
// slots from oldest to newest.
// Gram data: value a*kAndersonMax + c = dF_a . dF_c, value kAndersonMax^2 + a = dF_a . F_m.
template <typename T>
hipError_t launch_anderson_gram(const Geom& g, const T* Fbase, long long slot_stride,
                                const int* order, const int* m1, double* partials, int nred,
                                const int* active, hipStream_t st);
// out = G_m - sum_a gamma[b*kAndersonMax + a] (G_{a+1} - G_a)
template <typename T>
hipError_t launch_anderson_mix(const Geom& g, const T* Gbase, long long slot_stride,
                               const int* order, const int* m1, const double* gamma, T* out,
                               const int* active, hipStream_t st);

// number of lines along the load axis without a broken voxel, per RVE
template <typename T>
hipError_t launch_fracture_count(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* phi, double thr, int axis, int* count,
                                 const int* active, hipStream_t st);
// Hn = max(E_b^2 psi1 + psi_ini, Hn) (or without max)
template <typename T>
hipError_t launch_commit_history(const Geom& g, const T* psi1, const T* psi_ini, const double* E,
                                 int history, T* Hn, const int* active, hipStream_t st);
// zero n integers (a kernel, so that captured graphs hold no memset node)
hipError_t launch_zero_int(int* p, int n, hipStream_t st);

}  // namespace mirve
