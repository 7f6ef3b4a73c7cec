// Launchers of the monolithic Newton-Raphson step (Sec. 4.1, Eq. 22-31):
// one RVE per launch, FP64, fields offset to that RVE; a Newton vector is
// (x: s strain fields, phi, E), n = (s + 1) N + 1 values.
#pragma once
#include "kernels.h"

namespace mirve {

struct NrArgs {
    Geom g;
    const uint16_t* mat_id;
    const MatEntry<double>* mat;
    F6 f;                    // unit load (Mandel)
    const double* x;         // fluctuation strain of the Newton point
    double E;                // load of the Newton point
    const double* phi;       // damage of the Newton point
    const double* psi_ini;   // enrichment energy (Eq. 37a)
    const double* Hn;        // committed history
    int history;
};
// H = max(psi0 + psi_ini, Hn) at the Newton point
hipError_t launch_nr_history(const NrArgs& a, double* H, hipStream_t st);
// pointwise part of J dq: w (s fields, divided by g(0)), dphi copy, t2 = g' dH
hipError_t launch_nr_jac_point(const NrArgs& a, const double* dq, double inv_g0, double* w,
                               double* dphi_out, double* t2, hipStream_t st);
// out = (cx xs, ca a + cb b, escale * esrc[0] + eadd)
hipError_t launch_nr_pack(long long sN, long long N, double* out, const double* xs, double cx,
                          const double* a, double ca, const double* b, double cb,
                          const double* esrc, double escale, double eadd, hipStream_t st);
// blocks of the dot-product partials for vectors of length n (<= 64)
int nr_dot_blocks(long long n);
// out[j] = V_j . w for j < k (partials: k * nr_dot_blocks(n) doubles)
hipError_t launch_mdot(const double* V, long long ldv, int k, const double* w, long long n,
                       double* partials, double* out, hipStream_t st);
// w += alpha sum_{j<k} c[j] V_j (c on the device)
hipError_t launch_maxpy(const double* V, long long ldv, int k, const double* c, double alpha,
                        double* w, long long n, hipStream_t st);
// GMRES least-squares part on the device (one thread each): gv = sqrt(nrm2[0]) e_1;
// column j of the Hessenberg matrix (hA + hB, norm sqrt(hB[j + 1])) into R
// (column stride ldr) with its Givens rotation, est[j] = |residual| (NaN at
// a breakdown); y = R^-1 gv over k columns
hipError_t launch_gmres_start(double* gv, int m, const double* nrm2, hipStream_t st);
hipError_t launch_gmres_col(int j, int ldr, const double* hA, const double* hB, double* R, double* cs,
                            double* sn, double* gv, double* est, hipStream_t st);
hipError_t launch_gmres_solve(int k, int ldr, const double* R, const double* gv, double* y,
                              hipStream_t st);
// w /= sqrt(nrm2[0])
hipError_t launch_unit_scale(double* w, long long n, const double* nrm2, hipStream_t st);
// y = a x + b y
hipError_t launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st);
// x += alpha dx, phi += alpha dphi; out[0..3] = |dx + dE f|^2, |x + E_new f|^2,
// |dphi|^2, |phi|^2 (partials: 4 * nr_dot_blocks(N) doubles)
hipError_t launch_nr_update(int s, long long N, const double* dq, double alpha, const F6& f,
                            double E_new, double* x, double* phi, double* partials, double* out,
                            hipStream_t st);


}  // namespace mirve
