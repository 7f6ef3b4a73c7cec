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

constexpr int kNotDone = 0x7fffffff;

// Device-resident scalars of one Krylov solve (one per RVE).
//
// The kernels of iteration k receive k.  A kernel that needs a dot product
// adds the per-block partials of the launch that produced them itself, in a
// fixed order (every block gets the same bits), so no finalize launch sits
// between the passes.  `conv` is the iteration at which the solve stopped
// (kNotDone while it runs, -1 for an RVE outside the solve).  It is written
// by block 0 of the launch that decides to stop, and read as `conv <= k`:
// every block of that launch reaches the same decision from the same sums,
// whether it sees the old or the new value.  Values a launch writes for
// iteration k sit in slot k & 1, while that launch reads slot (k - 1) & 1.
struct CgDev {
    double rr_hist[2];   // r.r at iteration k in slot k & 1
    double rr;           // latest r.r (progress reports)
    double rr0;          // r.r at iteration 0
    double bn2;          // ||b||^2 (stopping reference)
    double tol2;         // tol^2
    int conv;            // iteration at which the solve stopped, kNotDone, or -1
    int status;          // 0 running, 1 converged, 2 breakdown / non-finite, 3 max iterations
    int max_it;          // < 0: timing run (alpha = 0, beta = 1/2, never stops)
    int pad;
};

// Preconditioned CG of the damage system (one per RVE).  The FFT
// preconditioner is 1 / (abar + bbar |d(xi)|^2) between two diagonal
// scalings.
struct PcgDev {
    double rz_hist[2];   // r.z at iteration k in slot k & 1
    double rr;           // latest r.r
    double rr0;          // r.r at iteration 0
    double bn2, tol2;
    double abar, bbar;
    int conv, status, max_it, pad;
};

// x-forward modes: XF_GREEN the linear law; XF_CG the CG direction update
// with the linear law; XF_PCG / XF_PCG0 the damage preconditioner;
// XF_SPLIT the volumetric tension / compression split (nonlinear), which
// also records whether tr(eps) > 0 per voxel; XF_CG_T the CG direction
// update with the split's tangent at the recorded flags.
enum { XF_GREEN = 0, XF_CG = 1, XF_PCG = 2, XF_PCG0 = 3, XF_SPLIT = 4, XF_CG_T = 5 };
enum { AX_FWD = 0, AX_INV = 1, AX_FWD_P_INV = 2, AX_FWD_M_INV = 3 };
enum { XI_STORE = 0, XI_CG = 1, XI_PCG = 2 };
enum { PRE_JACOBI = 0, PRE_FFT = 1 };

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
    T* r;                // XF_CG: residual; XF_PCG*: damage residual (updated in place)
    T* p;                // XF_CG: direction (updated in place)
    T* x;                // XF_PCG: damage iterate; XF_CG: solution (both updated in place)
    const T* pd;         // XF_PCG: damage direction
    const T* q;          // XF_PCG: A pd
    const T* sc;         // XF_PCG*: diagonal scaling of the preconditioner
    const CgDev* cg;     // XF_CG, XF_CG_T
    PcgDev* pcg;         // XF_PCG*
    uint8_t* tmask;      // XF_SPLIT: written; XF_CG_T: read (1 where tr eps > 0)
    const double* rr_part;   // XF_CG: r.r partials of the previous x-inverse ([B][nblocks])
    const double* pap_prev;  // XF_CG: p.Ap partials of the previous x-forward ([B][nblocks])
    const double* pq_part;   // XF_PCG: p.q partials, RVE b at pq_part + b * pq_stride
    long long pq_stride;
    int pq_n;
    int iter;
    const int* active;   // XF_GREEN: optional per-RVE mask
    cplx<T>* spec;
    double* partials;    // [B][nblocks]
    int rows_per_block;
    int nblocks;
    int threads;         // block size (multiple of 64, <= 256)
    int nt;              // Krylov modes: stream the voxel vectors with non-temporal loads / stores
};

template <typename T>
struct AxisArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    cplx<T>* spec;
    const CgDev* cg;     // skip RVE b when cg[b].conv <= iter
    const PcgDev* pcg;   // or pcg[b].conv <= iter; AX_FWD_M_INV takes abar, bbar here
    const T* dsq;        // AX_FWD_M_INV: |d_j(k)|^2 of x, y, z at offsets 0, n_x, n_x + n_y
    int iter;
    const int* active;   // or when active && !active[b]
    int contiguous;      // 1: y lines (stride 1); 0: z lines (stride n_y)
    int lines;           // lines per block (y pass) / y columns per block (z pass)
    int threads;         // block size (multiple of 64, <= 256)
    int block_only;      // 1: the block pass even where the one-wave y pass applies
    double* partials;    // norm pass: [B][nparts] partial sums of ||out||^2
    int nparts;          // norm pass: blocks per slot (the x-inverse pass's count)
    double nscale;       // norm pass: scale^2 / N of out = scale F^-1{P : F[sigma]}
};

template <typename T>
struct XinvArgs {
    Geom g;
    AxisPlan pl;
    const cplx<T>* tw;
    const cplx<T>* spec;
    T scale;             // multiplies the (normalised) inverse
    T* out;              // XI_STORE (may be null: norm only); XI_PCG: z
    T* r;                // XI_CG (updated); XI_PCG: read for r.z
    const T* sc;         // XI_PCG: diagonal scaling
    CgDev* cg;           // XI_CG
    const PcgDev* pcg;   // XI_PCG
    const double* pAp_part;  // XI_CG: p.Ap partials of the x-forward pass ([B][nblocks])
    int iter;
    const int* active;
    double* partials;    // [B][nblocks]
    int rows_per_block;
    int nblocks;
    int threads;         // block size (multiple of 64, <= 256)
    int nt;              // Krylov modes: stream the voxel vectors with non-temporal loads / stores
};

template <typename T>
hipError_t launch_xfwd(const XfwdArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_axis(const AxisArgs<T>& a, int mode, int maxb, dim3 grid, size_t lds,
                       hipStream_t st);
template <typename T>
hipError_t launch_xinv(const XinvArgs<T>& a, int mode, int maxb, size_t lds, hipStream_t st);
// ||scale F^-1{P : F[sigma]}||^2 partials from the x-forward spectrum alone
// (2D, 128-, 256- or 512-point y lines): a.partials, a.nparts per slot
template <typename T>
hipError_t launch_axis_norm(const AxisArgs<T>& a, hipStream_t st);

// ---------------------------------------------------------------------------
// finalize kernels (one block per RVE, fixed-order sums)
// ---------------------------------------------------------------------------

// CG partials are [B][n] (one per block of the pass that made them).
// rr_hist[0] = r.r, conv = 0 if already converged (else kNotDone, -1 when inactive)
hipError_t launch_cg_init(CgDev* cg, const double* prr, const double* pb, int n, int B,
                          double tol, int max_it, const int* active, hipStream_t st);
// sums[b*kMaxVals + v] = sum_k partials[(b*kMaxVals + v)*kRedBlocks + k], v < nv
hipError_t launch_sum_partials(const double* partials, int n, int nv, int B, double* sums,
                               const int* active, hipStream_t st);
// sums[b*kMaxVals + slot] = sum_k p[b*n + k]  (pass partials)
hipError_t launch_sum_rows(const double* p, int n, int B, double* sums, int slot, hipStream_t st);
// sums[b*kMaxVals] = max_k partials[(b*kMaxVals)*kRedBlocks + k]
hipError_t launch_max_partials(const double* partials, int n, int B, double* sums,
                               const int* active, hipStream_t st);

// Damage PCG partials use the kMaxVals layout above: value 0 p.q, 1 r.z,
// 2 r.r, 3 b.b, 4 the diagonal term a(x), 5 the gradient weight w(x).
// Sets bn2, tol2, conv, status, max_it and the FFT preconditioner constants
// abar = mean a(x), bbar = mean w(x).
hipError_t launch_pcg_fin_start(PcgDev* d, const double* partials, int n, int B, double tol,
                                int max_it, double inv_N, const int* active, hipStream_t st);

// ---------------------------------------------------------------------------
// pointwise / stencil kernels; `nred` blocks per RVE for reductions
// ---------------------------------------------------------------------------

struct F6 {
    double v[6];
};

// eps1 = f + x, sigma1 = g C eps1, psi1 (0 on notch voxels); partial sums of
// sigma1:f (value 0) and sigma1:sigma1 (value 1); eps1 / sig1 written if
// non-null.  split = 1: the volumetric split law and its tensile energy.
template <typename T>
hipError_t launch_unit_response(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const T* phi, const T* x, const F6& f, int split, T* psi1,
                                T* eps1, T* sig1, double* partials, int nred, const int* active,
                                hipStream_t st);
// Newton update of the split mechanics: x += dx; partials ||dx||^2 (value 0)
// and ||f + x||^2 (value 1) over the s components.
template <typename T>
hipError_t launch_newton_update(const Geom& g, T* x, const T* dx, const F6& f, double* partials,
                                int nred, const int* active, hipStream_t st);

// H = max(E_b^2 psi1 + psi_ini, Hn) (history) or E_b^2 psi1 + psi_ini; rhs = 2H.
template <typename T>
hipError_t launch_history(const Geom& g, const T* psi1, const T* psi_ini, const T* Hn,
                          const double* E, int history, T* H, T* rhs, const int* active,
                          hipStream_t st);

// Damage operator q = a(x) p + D^T (w(x) D p): mode 0 a = Gc/l + 2H (H may be
// null), w = Gc l; mode 1 a = 1, w = c (the enrichment smoothing).
// damage_diag: dinv = 1 / diag (Jacobi) or its square root (FFT scaling);
// partials of a(x) (value 4) and w(x) (value 5).
template <typename T>
hipError_t launch_damage_diag(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* H, int mode, double c, int sqrt_out, T* dinv,
                              double* partials, int nred, const int* active, hipStream_t st);
template <typename T>
hipError_t launch_pcg_matvec(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                             const T* H, int mode, double c, const T* p, T* q, double* partials,
                             int nred, const PcgDev* d, const int* active, hipStream_t st);
// r = b - Ax; partials r.(dinv r), r.r, b.b
template <typename T>
hipError_t launch_pcg_start(const Geom& g, const T* b, const T* Ax, const T* dinv, T* r,
                            double* partials, int nred, const int* active, hipStream_t st);
// Iteration k, step 1: r.z and r.r from the partials the previous step left
// (RVE b at rz_part + b * rz_stride, rz_n values; likewise r.r), the stopping
// test, beta = rz_k / rz_{k-1}; then the direction p_new = z + beta p_old
// evaluated at the voxel and its stencil neighbours (z = dinv r for Jacobi,
// the stored field zf for the FFT preconditioner), q = A p_new, partials p.q
// (value 0) from nblk blocks per RVE (nblk <= kRedBlocks).
template <typename T>
hipError_t launch_pcg_matvec_dir(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                 const T* H, int mode, double c, int pre, const T* r,
                                 const T* dinv, const T* zf, const T* p_old, T* p_new, T* q,
                                 const double* rz_part, long long rz_stride, int rz_n,
                                 const double* rr_part, long long rr_stride, int rr_n,
                                 double* partials, int nblk, PcgDev* d, int iter, hipStream_t st);
// Iteration k, step 2 (Jacobi): alpha = rz_k / p.q (n_pq partials),
// x += alpha p, r -= alpha q, partials r.(dinv r) (value 1) and r.r
// (value 2) from nred blocks.
template <typename T>
hipError_t launch_pcg_update(const Geom& g, PcgDev* d, T* x, T* r, const T* p, const T* q,
                             const T* dinv, double* partials, int n_pq, int nred, int iter,
                             hipStream_t st);

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
// iterative refinement of the damage balance (FP64 solution, bulk-type correction)
template <typename T>
hipError_t launch_ir_residual(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                              const T* psi1, const T* psi_ini, const T* Hn, const double* E,
                              int history, const double* phi64, T* r, double* partials, int nred,
                              const int* active, hipStream_t st);
template <typename T>
hipError_t launch_ir_update(double* phi64, const T* delta, T* phi, long long n, int B,
                            const int* active, hipStream_t st);
template <typename T>
hipError_t launch_widen(const T* phi, double* phi64, long long n, int B, const int* active,
                        hipStream_t st);
template <typename T>
hipError_t launch_dissipation64(const Geom& g, const uint16_t* mat_id, const MatEntry<T>* mat,
                                const double* phi64, double* partials, int nred, const int* active,
                                hipStream_t st);
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
