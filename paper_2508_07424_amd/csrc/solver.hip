// Host driver of the toughness solver and the C ABI (include/mirve.h).
//
// Per dissipation step (Eq. 16, Sec. 4.1) the driver runs a staggered
// fixed point with Anderson acceleration on the damage field:
//   (M) equilibrium for the unit load E = 1 at the current damage by
//       conjugate gradients on compatible strains (Fourier-Galerkin, Eq. 24
//       R1, Eq. 26); every iteration is three (2D) or five (3D) LDS-staged
//       FFT passes with the constitutive law fused into the first and the
//       CG update fused into the last; alpha and beta stay on the device.
//   (A) the load E with D(phi(E)) = tau (Eq. 16c) by safeguarded Newton;
//       phi(E) solves the damage balance with H(E) = max(E^2 psi_o1 +
//       psi_ini, H^n) (Eq. 16b, 38) by Jacobi-preconditioned CG on the
//       stencil form of the operator, dD/dE from the tangent system.
//   (U) relative changes of phi and E below tol end the step (Eq. 30).
// Then the step is committed (history Eq. 38, trapezoid Eq. 33) and the
// fracture point is tested.  Only scalars cross to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/mirve.h"
#include "kernels.h"

namespace mirve {

static const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// stiffness tables (host)
// ---------------------------------------------------------------------------

// 3D Mandel index pairs: xx, yy, zz, yz, xz, xy
static const int kPairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};

static void mandel_of_tensor(const double t[3][3], double v[6]) {
    const double s2 = std::sqrt(2.0);
    for (int a = 0; a < 6; ++a) {
        const int i = kPairs[a][0], j = kPairs[a][1];
        v[a] = (i == j) ? t[i][j] : s2 * t[i][j];
    }
}

static void tensor_of_mandel(const double v[6], double t[3][3]) {
    const double is2 = 1.0 / std::sqrt(2.0);
    for (int a = 0; a < 6; ++a) {
        const int i = kPairs[a][0], j = kPairs[a][1];
        const double val = (i == j) ? v[a] : v[a] * is2;
        t[i][j] = val;
        t[j][i] = val;
    }
}

// Q with mandel(R t R^T) = Q mandel(t); orthogonal.  C' = Q C Q^T.
static void mandel_rotation(double theta, double Q[6][6]) {
    const double c = std::cos(theta), s = std::sin(theta);
    const double R[3][3] = {{c, -s, 0.0}, {s, c, 0.0}, {0.0, 0.0, 1.0}};
    for (int b = 0; b < 6; ++b) {
        double e[6] = {0, 0, 0, 0, 0, 0};
        e[b] = 1.0;
        double t[3][3], u[3][3];
        tensor_of_mandel(e, t);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += R[i][k] * t[k][l] * R[j][l];
                u[i][j] = acc;
            }
        double v[6];
        mandel_of_tensor(u, v);
        for (int a = 0; a < 6; ++a) Q[a][b] = v[a];
    }
}

struct HostMat {
    double C[6][6];
    double K, Gc, drive;
};

static HostMat phase_entry(const rve_phase& ph, double theta, bool notch, double k_res) {
    HostMat m;
    double C[6][6] = {{0}};
    if (ph.kind == RVE_PHASE_ISO) {
        const double lam = ph.E * ph.nu / ((1.0 + ph.nu) * (1.0 - 2.0 * ph.nu));
        const double mu = ph.E / (2.0 * (1.0 + ph.nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) C[i][j] = lam + (i == j ? 2.0 * mu : 0.0);
        for (int a = 3; a < 6; ++a) C[a][a] = 2.0 * mu;
    } else {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) C[i][j] = (i == j) ? ph.C11 : ph.C12;
        for (int a = 3; a < 6; ++a) C[a][a] = 2.0 * ph.C44;
    }
    double Q[6][6];
    mandel_rotation(theta, Q);
    double QC[6][6];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += Q[a][k] * C[k][b];
            QC[a][b] = acc;
        }
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += QC[a][k] * Q[b][k];
            m.C[a][b] = acc;
        }
    double kb = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) kb += m.C[i][j];
    m.K = kb / 9.0;
    m.Gc = ph.Gc;
    m.drive = 1.0;
    if (notch) {
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) m.C[a][b] *= k_res;
        m.K *= k_res;
        m.drive = 0.0;
    }
    return m;
}

// ---------------------------------------------------------------------------
// FFT plans
// ---------------------------------------------------------------------------

static bool factorize(int N, AxisPlan& pl) {
    pl.N = N;
    pl.nst = 0;
    int n = N;
    std::vector<int> r;
    while (n % 8 == 0) { r.push_back(8); n /= 8; }
    while (n % 4 == 0) { r.push_back(4); n /= 4; }
    while (n % 2 == 0) { r.push_back(2); n /= 2; }
    for (int p : {3, 5, 7}) while (n % p == 0) { r.push_back(p); n /= p; }
    if (n != 1 || (int)r.size() > kMaxStages) return false;
    pl.min_rad = 8;
    for (size_t i = 0; i < r.size(); ++i) {
        pl.rad[i] = r[i];
        pl.min_rad = std::min(pl.min_rad, r[i]);
    }
    pl.nst = (int)r.size();
    if (pl.nst == 0) { pl.min_rad = 1; }
    return true;
}

static int round_maxb(long long need) {
    if (need <= 1) return 1;
    if (need <= 2) return 2;
    if (need <= 4) return 4;
    if (need <= 8) return 8;
    return -1;
}

constexpr size_t kLdsCap = 60 * 1024;

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct Layout {
    size_t total = 0;
    size_t off(size_t bytes) {
        const size_t o = total;
        total += (bytes + 255) & ~size_t(255);
        return o;
    }
};

}  // namespace mirve

using namespace mirve;

struct SolverBase {
    virtual ~SolverBase() {}
    virtual int set_microstructure(const uint16_t*, const rve_phase*, int, const double*,
                                   const uint8_t*, const uint8_t*, double) = 0;
    virtual int step(double dtau, rve_step_info* out) = 0;
    virtual int get_field(int which, double* host, size_t count) = 0;
    virtual int set_field(int which, const double* host, size_t count) = 0;
    virtual int apply_green(const double* eps, double* out) = 0;
    virtual int apply_green_device(const void* eps, void* out, int repeat) = 0;
    virtual int solve_mechanics(int* it, double* Sigma1) = 0;
    virtual int solve_damage(double E, double* D, int* it, int commit) = 0;
    virtual int dissipation(double* D, double* G) = 0;
    double E_c = 0, Sigma_c = 0, T_c = 0, tau_c = 0, tau0 = 0;
    int step_c = 0;
    bool fractured = false;
    bool ready = false;
    double V = 0, A_g = 0;
};

struct rve_handle_s {
    rve_config cfg;
    std::unique_ptr<SolverBase> impl;
    std::string err;
};

namespace mirve {

template <typename T>
struct Solver : SolverBase {
    rve_handle_s* hd;
    rve_config cfg;
    Geom g;
    AxisPlan plx, ply, plz;
    int RB = 2, nbx = 1, maxb_x = 1;
    int txy = 1, maxb_y = 1, txz = 1, maxb_z = 1;
    size_t lds_x = 0, lds_y = 0, lds_z = 0;
    int nred = 1;
    hipStream_t st;
    double min_gc = 0;
    int load_axis = 1;

    // device pointers
    T *phi_c, *phi_w, *Hn, *psi_ini, *phi_ini, *psi1, *H, *px, *pr, *pp, *pq, *pdinv, *pb, *tmp;
    T *x, *x_c, *r, *p;
    T* aF[kAndersonMax + 1];
    T* aG[kAndersonMax + 1];
    cplx<T>* spec;
    cplx<T>* tw;
    uint16_t* mat_id;
    MatEntry<T>* mat;
    double *partials, *cgpA, *cgpB, *sums;
    CgDev* cg;
    PcgDev* pcg;
    int* count;
    // pinned host mirrors
    CgDev* h_cg = nullptr;
    PcgDev* h_pcg = nullptr;
    double* h_sums = nullptr;
    int* h_count = nullptr;

    int greenops = 0;

    static size_t layout(const rve_config& c, const Geom& g, int nbx, Layout& L, Solver* s) {
        const size_t fN = sizeof(T) * g.N;
        const size_t sN = fN * g.s;
        const int m1 = std::max(0, std::min(c.anderson_depth, kAndersonMax)) + 1;
        T** single[] = {s ? &s->phi_c : nullptr, s ? &s->phi_w : nullptr, s ? &s->Hn : nullptr,
                        s ? &s->psi_ini : nullptr, s ? &s->phi_ini : nullptr, s ? &s->psi1 : nullptr,
                        s ? &s->H : nullptr, s ? &s->px : nullptr, s ? &s->pr : nullptr,
                        s ? &s->pp : nullptr, s ? &s->pq : nullptr, s ? &s->pdinv : nullptr,
                        s ? &s->pb : nullptr, s ? &s->tmp : nullptr};
        std::vector<size_t> offs;
        for (size_t i = 0; i < sizeof(single) / sizeof(single[0]); ++i) offs.push_back(L.off(fN));
        std::vector<size_t> aoffF, aoffG;
        for (int i = 0; i < m1; ++i) { aoffF.push_back(L.off(fN)); aoffG.push_back(L.off(fN)); }
        const size_t ox = L.off(sN), oxc = L.off(sN), orr = L.off(sN), op = L.off(sN);
        const size_t ospec = L.off(sizeof(cplx<T>) * g.s * g.Nspec);
        const size_t otw = L.off(sizeof(cplx<T>) * (g.nx + g.ny + g.nz));
        const size_t omid = L.off(sizeof(uint16_t) * g.N);
        const size_t omat = L.off(sizeof(MatEntry<T>) * std::max(1, c.max_materials));
        const size_t opart = L.off(sizeof(double) * 40 * kRedBlocks);
        const size_t ocgA = L.off(sizeof(double) * std::max(nbx, 1));
        const size_t ocgB = L.off(sizeof(double) * std::max(nbx, 1));
        const size_t osums = L.off(sizeof(double) * 64);
        const size_t ocg = L.off(sizeof(CgDev));
        const size_t opcg = L.off(sizeof(PcgDev));
        const size_t ocnt = L.off(sizeof(int) * 4);
        if (s) {
            char* base = (char*)s->ws;
            for (size_t i = 0; i < offs.size(); ++i) *single[i] = (T*)(base + offs[i]);
            for (int i = 0; i <= kAndersonMax; ++i) {
                s->aF[i] = i < m1 ? (T*)(base + aoffF[i]) : nullptr;
                s->aG[i] = i < m1 ? (T*)(base + aoffG[i]) : nullptr;
            }
            s->x = (T*)(base + ox);
            s->x_c = (T*)(base + oxc);
            s->r = (T*)(base + orr);
            s->p = (T*)(base + op);
            s->spec = (cplx<T>*)(base + ospec);
            s->tw = (cplx<T>*)(base + otw);
            s->mat_id = (uint16_t*)(base + omid);
            s->mat = (MatEntry<T>*)(base + omat);
            s->partials = (double*)(base + opart);
            s->cgpA = (double*)(base + ocgA);
            s->cgpB = (double*)(base + ocgB);
            s->sums = (double*)(base + osums);
            s->cg = (CgDev*)(base + ocg);
            s->pcg = (PcgDev*)(base + opcg);
            s->count = (int*)(base + ocnt);
        }
        return L.total;
    }

    void* ws = nullptr;

    // geometry and launch shapes from a configuration; false if unsupported
    static bool make_geom(const rve_config& c, Geom& g, AxisPlan& px, AxisPlan& py, AxisPlan& pz,
                          int& RB, int& nbx, int& maxb_x, size_t& lds_x, int& txy, int& maxb_y,
                          size_t& lds_y, int& txz, int& maxb_z, size_t& lds_z, std::string& why) {
        g.dim = c.dim;
        g.s = c.dim == 2 ? 3 : 6;
        g.nx = c.n[0];
        g.ny = c.n[1];
        g.nz = c.dim == 3 ? c.n[2] : 1;
        g.nxh = g.nx / 2 + 1;
        g.N = (long long)g.nx * g.ny * g.nz;
        g.Nspec = (long long)g.nxh * g.ny * g.nz;
        g.h = c.h;
        g.ell = c.ell;
        g.k_res = c.k_res;
        g.inv_N = 1.0 / double(g.N);
        if (!factorize(g.nx, px) || !factorize(g.ny, py) || !factorize(g.nz, pz)) {
            why = "grid sizes must be products of 2, 3, 5, 7 (<= 1024)";
            return false;
        }
        const size_t ce = sizeof(cplx<T>);
        // x passes: rows per block
        RB = std::max(2, std::min(16, 1024 / std::max(1, g.nx)));
        RB &= ~1;
        while (RB > 2 && (size_t)g.s * (RB / 2) * g.nx * ce > kLdsCap) RB -= 2;
        lds_x = (size_t)g.s * (RB / 2) * g.nx * ce;
        if (lds_x > kLdsCap) { why = "n_x too large for the LDS budget"; return false; }
        maxb_x = round_maxb(((long long)g.s * (RB / 2) * g.nx / px.min_rad + 255) / 256);
        while (maxb_x < 0 && RB > 2) {
            RB -= 2;
            maxb_x = round_maxb(((long long)g.s * (RB / 2) * g.nx / px.min_rad + 255) / 256);
            lds_x = (size_t)g.s * (RB / 2) * g.nx * ce;
        }
        if (maxb_x < 0) { why = "x plan does not fit"; return false; }
        const int nrows = g.ny * g.nz;
        nbx = (nrows + RB - 1) / RB;
        auto pick_tx = [&](const AxisPlan& pl, int& tx, int& mb, size_t& lds) -> bool {
            for (int t : {8, 4, 2, 1}) {
                if (t > g.nxh && t > 1) continue;
                const size_t l = (size_t)g.s * t * pl.N * ce;
                const int m = round_maxb(((long long)g.s * t * pl.N / pl.min_rad + 255) / 256);
                if (l <= kLdsCap && m > 0) { tx = t; mb = m; lds = l; return true; }
            }
            return false;
        };
        if (!pick_tx(py, txy, maxb_y, lds_y)) { why = "n_y too large for the LDS budget"; return false; }
        if (g.dim == 3 && !pick_tx(pz, txz, maxb_z, lds_z)) {
            why = "n_z too large for the LDS budget";
            return false;
        }
        return true;
    }

    Solver(rve_handle_s* h, const rve_config& c, void* wsp, hipStream_t s) : hd(h), cfg(c), st(s) {
        std::string why;
        make_geom(c, g, plx, ply, plz, RB, nbx, maxb_x, lds_x, txy, maxb_y, lds_y, txz, maxb_z,
                  lds_z, why);
        ws = wsp;
        Layout L;
        layout(c, g, nbx, L, this);
        nred = (int)std::min<long long>((g.N + 255) / 256, kRedBlocks);
        int ax = 0;
        double best = -1;
        for (int a = 0; a < g.dim; ++a)
            if (std::fabs(c.f[a]) > best) { best = std::fabs(c.f[a]); ax = a; }
        load_axis = ax;
        V = double(g.N) * std::pow(g.h, g.dim);
    }

    ~Solver() override {
        if (h_cg) (void)hipHostFree(h_cg);
        if (h_pcg) (void)hipHostFree(h_pcg);
        if (h_sums) (void)hipHostFree(h_sums);
        if (h_count) (void)hipHostFree(h_count);
    }

    int fail(int code, const std::string& m) {
        hd->err = m;
        return code;
    }

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(RVE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

    int init_device() {
        HIPCHK(hipHostMalloc((void**)&h_cg, sizeof(CgDev), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_pcg, sizeof(PcgDev), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_sums, sizeof(double) * 64, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_count, sizeof(int) * 4, hipHostMallocDefault));
        // twiddles, exp(-2 pi i m / N), computed in long double
        std::vector<cplx<T>> t;
        for (int N : {g.nx, g.ny, g.nz}) {
            for (int m = 0; m < N; ++m) {
                const long double a = -2.0L * 3.141592653589793238462643383279502884L * m / N;
                t.push_back({T(std::cos(a)), T(std::sin(a))});
            }
        }
        plx.tw_off = 0;
        ply.tw_off = g.nx;
        plz.tw_off = g.nx + g.ny;
        HIPCHK(hipMemcpyAsync(tw, t.data(), t.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, st));
        HIPCHK(launch_fill<T>(x, T(0), g.s * g.N, st));
        HIPCHK(launch_fill<T>(x_c, T(0), g.s * g.N, st));
        HIPCHK(hipStreamSynchronize(st));
        return RVE_OK;
    }

    int sync() {
        HIPCHK(hipStreamSynchronize(st));
        return RVE_OK;
    }

    // ---- host <-> device field copies -----------------------------------
    int upload(T* dst, const double* src, size_t n) {
        if (sizeof(T) == sizeof(double)) {
            HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st));
        } else {
            std::vector<T> tmpv(n);
            for (size_t i = 0; i < n; ++i) tmpv[i] = T(src[i]);
            HIPCHK(hipMemcpyAsync(dst, tmpv.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        return RVE_OK;
    }
    int download(double* dst, const T* src, size_t n) {
        if (sizeof(T) == sizeof(double)) {
            HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        } else {
            std::vector<T> tmpv(n);
            HIPCHK(hipMemcpyAsync(tmpv.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (size_t i = 0; i < n; ++i) dst[i] = double(tmpv[i]);
        }
        return RVE_OK;
    }
    int read_sums(int nv) {
        HIPCHK(hipMemcpyAsync(h_sums, sums, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return RVE_OK;
    }

    // ---- Green operator passes --------------------------------------------
    int fwd_x(int mode, const T* phi, const T* eps, double fcoef, double* part) {
        XfwdArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.pl = plx;
        a.tw = tw + plx.tw_off;
        a.mat_id = mat_id;
        a.mat = mat;
        a.phi = phi;
        a.eps = eps;
        a.fcoef = T(fcoef);
        for (int c = 0; c < 6; ++c) a.f[c] = T(c < g.s ? cfg.f[c] : 0.0);
        a.r = r;
        a.p = p;
        a.cg = cg;
        a.spec = spec;
        a.partials = part;
        a.rows_per_block = RB;
        HIPCHK(launch_xfwd<T>(a, mode, maxb_x, nbx, lds_x, st));
        return RVE_OK;
    }
    int axes(const CgDev* c) {
        AxisArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.spec = spec;
        a.cg = c;
        if (g.dim == 2) {
            a.pl = ply;
            a.tw = tw + ply.tw_off;
            a.axis = 1;
            a.tx = txy;
            HIPCHK(launch_axis<T>(a, AX_FWD_P_INV, maxb_y, dim3((g.nxh + txy - 1) / txy, g.nz),
                                  lds_y, st));
        } else {
            a.pl = ply;
            a.tw = tw + ply.tw_off;
            a.axis = 1;
            a.tx = txy;
            const dim3 gy((g.nxh + txy - 1) / txy, g.nz);
            HIPCHK(launch_axis<T>(a, AX_FWD, maxb_y, gy, lds_y, st));
            AxisArgs<T> b = a;
            b.pl = plz;
            b.tw = tw + plz.tw_off;
            b.axis = 2;
            b.tx = txz;
            HIPCHK(launch_axis<T>(b, AX_FWD_P_INV, maxb_z, dim3((g.nxh + txz - 1) / txz, g.ny),
                                  lds_z, st));
            HIPCHK(launch_axis<T>(a, AX_INV, maxb_y, gy, lds_y, st));
        }
        return RVE_OK;
    }
    int inv_x(int mode, T* out, double scale, double* part) {
        XinvArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.pl = plx;
        a.tw = tw + plx.tw_off;
        a.spec = spec;
        a.scale = T(scale);
        a.out = out;
        a.x = x;
        a.p = p;
        a.r = r;
        a.cg = mode == XI_CG ? cg : nullptr;
        a.partials = part;
        a.rows_per_block = RB;
        HIPCHK(launch_xinv<T>(a, mode, maxb_x, nbx, lds_x, st));
        return RVE_OK;
    }
#define CHK(expr)                    \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != RVE_OK) return rc_; \
    } while (0)

    // out = scale * F^-1{P : F[g C (eps + fcoef f)]}; ||out||^2 partials in part
    int green(const T* phi, const T* eps, double fcoef, T* out, double scale, double* part) {
        CHK(fwd_x(XF_GREEN, phi, eps, fcoef, part));
        CHK(axes(nullptr));
        CHK(inv_x(XI_STORE, out, scale, part));
        ++greenops;
        return RVE_OK;
    }

    // ---- (M) mechanics CG ---------------------------------------------------
    int mech_solve(const T* phi, int* iters) {
        CHK(green(phi, nullptr, 1.0, nullptr, 1.0, cgpB));          // ||b||^2
        CHK(green(phi, x, 1.0, r, -1.0, cgpA));                     // r0 = -P[gC(f + x)]
        HIPCHK(launch_cg_init(cg, cgpA, nbx, cgpB, nbx, cfg.tol_cg, cfg.max_cg, st));
        int chunk = 8;
        int total = 0;
        for (;;) {
            for (int k = 0; k < chunk; ++k) {
                CHK(fwd_x(XF_CG, phi, nullptr, 0.0, cgpA));
                CHK(axes(cg));
                HIPCHK(launch_cg_alpha(cg, cgpA, nbx, st));
                CHK(inv_x(XI_CG, nullptr, 1.0, cgpB));
                HIPCHK(launch_cg_beta(cg, cgpB, nbx, st));
            }
            total += chunk;
            HIPCHK(hipMemcpyAsync(h_cg, cg, sizeof(CgDev), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (h_cg->done) break;
            if (total > cfg.max_cg + chunk) break;
            chunk = std::min(chunk * 2, 64);
        }
        greenops += h_cg->it;
        if (iters) *iters = h_cg->it;
        if (h_cg->status == 1) return RVE_OK;
        if (h_cg->status == 2) {
            // a breakdown at a residual already near the target is convergence
            if (std::isfinite(h_cg->rr) && h_cg->rr <= 1e4 * h_cg->tol2 * h_cg->bn2) return RVE_OK;
            return fail(RVE_ENUMERIC, "mechanics CG breakdown or non-finite residual");
        }
        return fail(RVE_ENOCONV, "mechanics CG did not converge");
    }

    int unit_response(const T* phi, double* Sigma1, double* sig2, T* eps1 = nullptr,
                      T* sig1 = nullptr) {
        HIPCHK(launch_unit_response<T>(g, mat_id, mat, phi, x, cfg.f, cfg.split, psi1, eps1, sig1,
                                       partials, nred, st));
        HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, 2, sums, st));
        CHK(read_sums(2));
        if (Sigma1) *Sigma1 = h_sums[0] / double(g.N);
        if (sig2) *sig2 = h_sums[1];
        if (!std::isfinite(h_sums[0])) return fail(RVE_ENUMERIC, "non-finite unit stress");
        return RVE_OK;
    }

    // ---- (A) damage PCG -----------------------------------------------------
    // Solve a(x) u + D^T(w D u) = b (mode 0: a = Gc/l + 2 Hc, w = Gc l; mode 1:
    // a = 1, w = c) from the initial guess in u.
    int pcg_solve(const T* Hc, int mode, double c, const T* b, T* u, double tol, int max_it,
                  int* iters) {
        HIPCHK(launch_damage_diag<T>(g, mat_id, mat, Hc, mode, c, pdinv, st));
        HIPCHK(launch_pcg_matvec<T>(g, mat_id, mat, Hc, mode, c, u, pq, nullptr, nred, nullptr, st));
        HIPCHK(launch_pcg_start<T>(g, b, pq, pdinv, pr, pp, partials, nred, st));
        HIPCHK(launch_pcg_fin_start(pcg, partials, nred, tol, max_it, st));
        int chunk = 8, total = 0;
        for (;;) {
            for (int k = 0; k < chunk; ++k) {
                HIPCHK(launch_pcg_matvec<T>(g, mat_id, mat, Hc, mode, c, pp, pq, partials, nred,
                                            pcg, st));
                HIPCHK(launch_pcg_fin_alpha(pcg, partials, nred, st));
                HIPCHK(launch_pcg_update<T>(g, pcg, u, pr, pp, pq, pdinv, partials, nred, st));
                HIPCHK(launch_pcg_fin_beta(pcg, partials, nred, st));
                HIPCHK(launch_pcg_dir<T>(g, pcg, pr, pdinv, pp, st));
            }
            total += chunk;
            HIPCHK(hipMemcpyAsync(h_pcg, pcg, sizeof(PcgDev), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (h_pcg->done) break;
            if (total > max_it + chunk) break;
            chunk = std::min(chunk * 2, 64);
        }
        if (iters) *iters += h_pcg->it;
        if (h_pcg->status == 1) return RVE_OK;
        if (h_pcg->status == 2) {
            if (std::isfinite(h_pcg->rr) && h_pcg->rr <= 1e4 * h_pcg->tol2 * h_pcg->bn2) return RVE_OK;
            if (h_pcg->bn2 == 0.0) return RVE_OK;
            return fail(RVE_ENUMERIC, "damage PCG breakdown or non-finite residual");
        }
        return fail(RVE_ENOCONV, "damage PCG did not converge");
    }

    int dissip(const T* phi, double* D, double* G) {
        HIPCHK(launch_dissipation<T>(g, mat_id, mat, phi, partials, nred, st));
        HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, 2, sums, st));
        CHK(read_sums(2));
        const double hd_ = std::pow(g.h, g.dim);
        if (D) *D = h_sums[0] * hd_;
        if (G) *G = h_sums[1] * hd_;
        if (!std::isfinite(h_sums[0])) return fail(RVE_ENUMERIC, "non-finite dissipation");
        return RVE_OK;
    }

    // phi(E) into u (warm start in u); D(phi(E)) out
    int damage_at(double E, T* u, double* D, int* npcg) {
        HIPCHK(launch_history<T>(g, psi1, psi_ini, Hn, E, cfg.history, H, st));
        HIPCHK(launch_scaled<T>(H, 2.0, pb, g.N, st));
        CHK(pcg_solve(H, 0, 0.0, pb, u, cfg.tol_pcg, cfg.max_pcg, npcg));
        return dissip(u, D, nullptr);
    }

    // dD/dE at (E, u = phi(E)) via the tangent system with the same H
    int damage_slope(double E, const T* u, double* dD, int* npcg) {
        HIPCHK(launch_tangent_rhs<T>(g, u, psi1, psi_ini, Hn, E, cfg.history, pb, st));
        HIPCHK(launch_fill<T>(tmp, T(0), g.N, st));
        CHK(pcg_solve(H, 0, 0.0, pb, tmp, cfg.tol_pcg, cfg.max_pcg, npcg));
        HIPCHK(launch_dissipation_dir<T>(g, mat_id, mat, u, tmp, partials, nred, st));
        HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, 1, sums, st));
        CHK(read_sums(1));
        *dD = h_sums[0] * std::pow(g.h, g.dim);
        return RVE_OK;
    }

    int max_psi1(double* m) {
        HIPCHK(launch_max_field<T>(psi1, g.N, partials, nred, st));
        HIPCHK(launch_max_partials(partials, nred, sums, st));
        CHK(read_sums(1));
        *m = h_sums[0];
        return RVE_OK;
    }

    // E >= 0 with D(phi(E)) = tau (Eq. 16c); phi(E) left in u.
    int arclength(double tau, double E0, double* Eout, T* u, int* npcg) {
        double lo = 0.0, hi = INFINITY;
        double E = E0;
        if (!(E > 0.0)) {
            double pm = 0.0;
            CHK(max_psi1(&pm));
            E = pm > 0.0 ? std::sqrt(min_gc / cfg.ell / pm) : 1.0;
        }
        for (int it = 0; it < 200; ++it) {
            double Dv = 0.0;
            CHK(damage_at(E, u, &Dv, npcg));
            if (std::fabs(Dv - tau) <= cfg.tol_al * tau) { *Eout = E; return RVE_OK; }
            if (Dv < tau) lo = std::max(lo, E);
            else hi = std::min(hi, E);
            double dD = 0.0;
            CHK(damage_slope(E, u, &dD, npcg));
            double En = dD > 0.0 ? E - (Dv - tau) / dD : NAN;
            if (!(lo < En && En < hi)) En = std::isinf(hi) ? 2.0 * E : 0.5 * (lo + hi);
            if (!std::isinf(hi) && hi - lo <= 1e-15 * hi) { *Eout = E; return RVE_OK; }
            E = En;
        }
        return fail(RVE_ENOCONV, "dissipation constraint (arc-length) did not converge");
    }

    // ---- Anderson mixing (host side of the small least-squares problem) -------
    int anderson_mix(int count, int m1_max, T* out) {
        const int m1 = std::min(count, m1_max);
        Ptrs<T> F, G;
        for (int i = 0; i < m1; ++i) {
            const int slot = (count - m1 + i) % m1_max;
            F.p[i] = aF[slot];
            G.p[i] = aG[slot];
        }
        for (int i = m1; i <= kAndersonMax; ++i) { F.p[i] = F.p[0]; G.p[i] = G.p[0]; }
        HIPCHK(launch_anderson_gram<T>(g, F, m1, partials, nred, st));
        const int nv = kAndersonMax * kAndersonMax + kAndersonMax;
        HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, nv, sums, st));
        CHK(read_sums(nv));
        const int m = m1 - 1;
        // normal equations (dF^T dF + ridge) gamma = dF^T F_m
        double A[kAndersonMax][kAndersonMax], bvec[kAndersonMax];
        double tr = 0.0;
        for (int a = 0; a < m; ++a) tr += h_sums[a * kAndersonMax + a];
        for (int a = 0; a < m; ++a) {
            for (int b = 0; b < m; ++b) A[a][b] = h_sums[a * kAndersonMax + b];
            A[a][a] += 1e-14 * tr;
            bvec[a] = h_sums[kAndersonMax * kAndersonMax + a];
        }
        // Gaussian elimination with partial pivoting
        for (int k = 0; k < m; ++k) {
            int piv = k;
            for (int i = k + 1; i < m; ++i)
                if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
            if (piv != k) {
                for (int j = 0; j < m; ++j) std::swap(A[k][j], A[piv][j]);
                std::swap(bvec[k], bvec[piv]);
            }
            if (A[k][k] == 0.0) return fail(RVE_ENUMERIC, "singular Anderson system");
            for (int i = k + 1; i < m; ++i) {
                const double f = A[i][k] / A[k][k];
                for (int j = k; j < m; ++j) A[i][j] -= f * A[k][j];
                bvec[i] -= f * bvec[k];
            }
        }
        Coef c;
        for (int i = 0; i < kAndersonMax; ++i) c.v[i] = 0.0;
        for (int k = m - 1; k >= 0; --k) {
            double s = bvec[k];
            for (int j = k + 1; j < m; ++j) s -= A[k][j] * c.v[j];
            c.v[k] = s / A[k][k];
        }
        for (int k = 0; k < m; ++k)
            if (!std::isfinite(c.v[k])) return fail(RVE_ENUMERIC, "non-finite Anderson weights");
        HIPCHK(launch_anderson_mix<T>(g, G, m1, c, out, st));
        return RVE_OK;
    }

    // ---- microstructure ----------------------------------------------------
    int set_microstructure(const uint16_t* pid, const rve_phase* phases, int nph,
                           const double* theta, const uint8_t* vmask, const uint8_t* disc,
                           double phi_M) override {
        if (!pid || !phases || nph <= 0) return fail(RVE_EINVAL, "phase_id and phases required");
        if (!(phi_M > 0.0 && phi_M < 1.0)) return fail(RVE_EINVAL, "phi_M must be in (0, 1)");
        for (int i = 0; i < nph; ++i) {
            const rve_phase& ph = phases[i];
            if (!(ph.Gc > 0.0) || !std::isfinite(ph.Gc)) return fail(RVE_EINVAL, "Gc must be > 0");
            if (ph.kind == RVE_PHASE_ISO) {
                if (!(ph.E > 0.0) || !(ph.nu > -1.0 && ph.nu < 0.5))
                    return fail(RVE_EINVAL, "isotropic phase needs E > 0, -1 < nu < 0.5");
            } else if (ph.kind == RVE_PHASE_CUBIC) {
                if (!(ph.C11 > std::fabs(ph.C12)) || !(ph.C11 + 2 * ph.C12 > 0) || !(ph.C44 > 0))
                    return fail(RVE_EINVAL, "cubic phase is not positive definite");
            } else {
                return fail(RVE_EINVAL, "unknown phase kind");
            }
        }
        std::map<std::tuple<int, double, int>, int> keys;
        std::vector<uint16_t> ids(g.N);
        std::vector<MatEntry<T>> table;
        min_gc = INFINITY;
        for (long long i = 0; i < g.N; ++i) {
            const int ph = pid[i];
            if (ph >= nph) return fail(RVE_EINVAL, "phase_id out of range");
            const double th = theta ? theta[i] : 0.0;
            if (!std::isfinite(th)) return fail(RVE_EINVAL, "non-finite theta");
            const int nt = vmask ? (vmask[i] ? 1 : 0) : 0;
            auto key = std::make_tuple(ph, phases[ph].kind == RVE_PHASE_ISO ? 0.0 : th, nt);
            auto it = keys.find(key);
            int id;
            if (it == keys.end()) {
                id = (int)table.size();
                if (id >= cfg.max_materials || id >= kMaxMat)
                    return fail(RVE_EINVAL, "more distinct materials than max_materials");
                keys[key] = id;
                HostMat hm = phase_entry(phases[ph], std::get<1>(key), nt != 0, cfg.k_res);
                MatEntry<T> me;
                std::memset(&me, 0, sizeof(me));
                static const int in2d[3] = {0, 1, 5};
                for (int a = 0; a < g.s; ++a)
                    for (int b = 0; b < g.s; ++b) {
                        const int ia = g.dim == 2 ? in2d[a] : a;
                        const int ib = g.dim == 2 ? in2d[b] : b;
                        me.C[a * g.s + b] = T(hm.C[ia][ib]);
                    }
                me.K = T(hm.K);
                me.Gc = T(hm.Gc);
                me.drive = T(hm.drive);
                table.push_back(me);
            } else {
                id = it->second;
            }
            ids[i] = (uint16_t)id;
            min_gc = std::min(min_gc, phases[ph].Gc);
        }
        HIPCHK(hipMemcpyAsync(mat_id, ids.data(), sizeof(uint16_t) * g.N, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(mat, table.data(), sizeof(MatEntry<T>) * table.size(),
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        // reference crack area: lines along the load axis without a notch voxel
        if (cfg.A_g > 0) {
            A_g = cfg.A_g;
        } else {
            long long lines = 0;
            const int la = load_axis;
            const int n0 = g.nx, n1 = g.ny, n2 = g.nz;
            const int len = la == 0 ? n0 : la == 1 ? n1 : n2;
            const long long nl = g.N / len;
            for (long long l = 0; l < nl; ++l) {
                long long base, stride;
                if (la == 0) { base = l * n0; stride = 1; }
                else if (la == 1) { base = (l / n0) * (long long)n0 * n1 + (l % n0); stride = n0; }
                else { base = l; stride = (long long)n0 * n1; }
                bool notch = false;
                for (int k = 0; k < len && vmask; ++k)
                    if (vmask[base + k * stride]) { notch = true; break; }
                if (!notch) ++lines;
            }
            A_g = double(lines) * std::pow(g.h, g.dim - 1);
        }
        // crack-tip enrichment (Eq. 35): (1 + l^2 D^T D) phi_o = phi_disc
        bool any = false;
        std::vector<double> d(g.N, 0.0);
        if (disc)
            for (long long i = 0; i < g.N; ++i)
                if (disc[i]) { d[i] = 1.0; any = true; }
        if (any) {
            CHK(upload(pb, d.data(), g.N));
            HIPCHK(launch_fill<T>(phi_ini, T(0), g.N, st));
            int it = 0;
            const double ctol = sizeof(T) == 8 ? 1e-15 : 1e-7;
            CHK(pcg_solve(nullptr, 1, cfg.ell * cfg.ell, pb, phi_ini, ctol, 100000, &it));
            HIPCHK(launch_max_field<T>(phi_ini, g.N, partials, nred, st));
            HIPCHK(launch_max_partials(partials, nred, sums, st));
            HIPCHK(launch_scale_field<T>(phi_ini, sums, phi_M, g.N, st));
        } else {
            HIPCHK(launch_fill<T>(phi_ini, T(0), g.N, st));
        }
        HIPCHK(launch_psi_ini<T>(g, mat_id, mat, phi_ini, psi_ini, st));
        HIPCHK(launch_copy<T>(phi_ini, phi_c, g.N, st));
        HIPCHK(launch_copy<T>(psi_ini, Hn, g.N, st));
        HIPCHK(launch_fill<T>(x, T(0), g.s * g.N, st));
        HIPCHK(launch_fill<T>(x_c, T(0), g.s * g.N, st));
        HIPCHK(launch_fill<T>(psi1, T(0), g.N, st));
        double D0 = 0.0;
        CHK(dissip(phi_c, &D0, nullptr));
        tau_c = tau0 = D0;
        E_c = Sigma_c = T_c = 0.0;
        step_c = 0;
        fractured = false;
        ready = true;
        return RVE_OK;
    }

    // ---- one step ------------------------------------------------------------
    int step(double dtau, rve_step_info* out) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(RVE_EINVAL, "dtau must be > 0");
        int rc = step_impl(dtau, out);
        if (rc != RVE_OK) {
            // transactional: the working strain restarts from the committed one
            (void)launch_copy<T>(x_c, x, g.s * g.N, st);
            (void)hipStreamSynchronize(st);
        }
        return rc;
    }

    int step_impl(double dtau, rve_step_info* out) {
        const double tau = tau_c + dtau;
        greenops = 0;
        int ncg = 0, npcg = 0;
        HIPCHK(launch_copy<T>(phi_c, phi_w, g.N, st));
        HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, st));
        double E = E_c;
        const int m1_max = std::max(0, std::min(cfg.anderson_depth, kAndersonMax)) + 1;
        int nhist = 0;
        bool conv = false;
        int it = 0;
        for (it = 1; it <= cfg.max_stagger; ++it) {
            int c = 0;
            CHK(mech_solve(phi_w, &c));
            ncg += c;
            CHK(unit_response(phi_w, nullptr, nullptr));
            HIPCHK(launch_copy<T>(phi_w, px, g.N, st));
            double En = 0.0;
            CHK(arclength(tau, E, &En, px, &npcg));
            HIPCHK(launch_diff_norms<T>(px, phi_w, g.N, partials, nred, st));
            HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, 2, sums, st));
            CHK(read_sums(2));
            const double dphi = std::sqrt(h_sums[0]) / std::max(std::sqrt(h_sums[1]), 1e-300);
            const double dE = std::fabs(En - E) / std::max(std::fabs(En), 1e-300);
            const double err = std::max(dphi, dE);
            if (!std::isfinite(err)) return fail(RVE_ENUMERIC, "non-finite stagger update");
            E = En;
            if (err < cfg.tol) {
                HIPCHK(launch_copy<T>(px, phi_w, g.N, st));
                conv = true;
                break;
            }
            if (m1_max > 1) {
                const int slot = nhist % m1_max;
                HIPCHK(launch_sub<T>(px, phi_w, aF[slot], g.N, st));
                HIPCHK(launch_copy<T>(px, aG[slot], g.N, st));
                ++nhist;
                if (nhist >= 2) {
                    CHK(anderson_mix(nhist, m1_max, phi_w));
                } else {
                    HIPCHK(launch_copy<T>(px, phi_w, g.N, st));
                }
            } else {
                HIPCHK(launch_copy<T>(px, phi_w, g.N, st));
            }
        }
        if (!conv) return fail(RVE_ENOCONV, "stagger did not converge");
        // final equilibrium at the committed damage, then commit
        int c = 0;
        CHK(mech_solve(phi_w, &c));
        ncg += c;
        double Sigma1 = 0.0, s2 = 0.0;
        CHK(unit_response(phi_w, &Sigma1, &s2));
        // residuals of the committed state: R1 (equilibrium) and R2 (damage with the H
        // used by the last damage solve)
        CHK(green(phi_w, x, 1.0, nullptr, 1.0, cgpB));
        HIPCHK(launch_sum_partials(cgpB, 0, nbx, 1, sums, st));
        CHK(read_sums(1));
        const double R1 = std::sqrt(h_sums[0]) / std::max(std::sqrt(s2), 1e-300);
        HIPCHK(launch_damage_residual<T>(g, mat_id, mat, H, phi_w, partials, nred, st));
        HIPCHK(launch_sum_partials(partials, kRedBlocks, nred, 2, sums, st));
        CHK(read_sums(2));
        const double R2 = std::sqrt(h_sums[0]) / std::max(std::sqrt(h_sums[1]), 1e-300);
        HIPCHK(launch_commit_history<T>(g, psi1, psi_ini, E, cfg.history, Hn, st));
        HIPCHK(launch_copy<T>(phi_w, phi_c, g.N, st));
        HIPCHK(launch_copy<T>(x, x_c, g.s * g.N, st));
        const double Sigma = E * Sigma1;
        T_c += 0.5 * (Sigma + Sigma_c) * (E - E_c);
        E_c = E;
        Sigma_c = Sigma;
        tau_c = tau;
        ++step_c;
        double D = 0.0, G = 0.0;
        CHK(dissip(phi_c, &D, &G));
        HIPCHK(hipMemsetAsync(count, 0, sizeof(int), st));
        HIPCHK(launch_fracture_count<T>(g, mat_id, mat, phi_c, cfg.frac_threshold, load_axis, count, st));
        HIPCHK(hipMemcpyAsync(h_count, count, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        fractured = h_count[0] == 0;
        if (out) {
            out->E = E;
            out->Sigma = Sigma;
            out->D = D;
            out->Gamma = G;
            out->tau = tau;
            out->T = T_c;
            out->n_stagger = it;
            out->n_cg = ncg;
            out->n_pcg = npcg;
            out->n_greenop = greenops;
            out->res_R1 = R1;
            out->res_R2 = R2;
            out->res_R3 = std::fabs(D - tau) / tau;
            out->fractured = fractured ? 1 : 0;
            out->step = step_c;
        }
        return RVE_OK;
    }

    // ---- fields ------------------------------------------------------------------
    int get_field(int which, double* hostp, size_t cnt) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        const size_t N = (size_t)g.N, sN = (size_t)g.s * g.N;
        switch (which) {
            case RVE_FIELD_PHI: if (cnt != N) break; return download(hostp, phi_c, N);
            case RVE_FIELD_HIST: if (cnt != N) break; return download(hostp, Hn, N);
            case RVE_FIELD_PSI_INI: if (cnt != N) break; return download(hostp, psi_ini, N);
            case RVE_FIELD_PSI1: if (cnt != N) break; return download(hostp, psi1, N);
            case RVE_FIELD_PHI_INI: if (cnt != N) break; return download(hostp, phi_ini, N);
            case RVE_FIELD_EPS1:
            case RVE_FIELD_SIG1: {
                if (cnt != sN) break;
                CHK(unit_response(phi_c, nullptr, nullptr, r, p));
                return download(hostp, which == RVE_FIELD_EPS1 ? r : p, sN);
            }
            default: return fail(RVE_EINVAL, "unknown field");
        }
        return fail(RVE_EINVAL, "field size mismatch");
    }

    int set_field(int which, const double* hostp, size_t cnt) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        const size_t N = (size_t)g.N;
        if (cnt != N) return fail(RVE_EINVAL, "field size mismatch");
        for (size_t i = 0; i < N; ++i)
            if (!std::isfinite(hostp[i])) return fail(RVE_EINVAL, "non-finite field value");
        switch (which) {
            case RVE_FIELD_PHI: CHK(upload(phi_c, hostp, N)); return sync();
            case RVE_FIELD_HIST: CHK(upload(Hn, hostp, N)); return sync();
            case RVE_FIELD_PSI1: CHK(upload(psi1, hostp, N)); return sync();
            default: return fail(RVE_EINVAL, "field is read-only");
        }
    }

    int apply_green(const double* eps, double* outp) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        const size_t sN = (size_t)g.s * g.N;
        CHK(upload(r, eps, sN));
        CHK(green(phi_c, r, 0.0, p, 1.0, cgpB));
        return download(outp, p, sN);
    }

    int apply_green_device(const void* eps, void* outp, int repeat) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        for (int i = 0; i < repeat; ++i)
            CHK(green(phi_c, (const T*)eps, 0.0, (T*)outp, 1.0, cgpB));
        return RVE_OK;
    }

    int solve_mechanics(int* it, double* Sigma1) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, st));
        CHK(mech_solve(phi_c, it));
        CHK(unit_response(phi_c, Sigma1, nullptr));
        HIPCHK(launch_copy<T>(x, x_c, g.s * g.N, st));
        return sync();
    }

    int solve_damage(double E, double* D, int* it, int commit) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        HIPCHK(launch_copy<T>(phi_c, px, g.N, st));
        int n = 0;
        CHK(damage_at(E, px, D, &n));
        if (it) *it = n;
        if (commit) HIPCHK(launch_copy<T>(px, phi_c, g.N, st));
        return sync();
    }

    int dissipation(double* D, double* G) override {
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        return dissip(phi_c, D, G);
    }
};

}  // namespace mirve

// ===========================================================================
// C ABI
// ===========================================================================

static int validate(const rve_config* c, std::string& why) {
    if (!c) { why = "null config"; return RVE_EINVAL; }
    if (c->dim != 2 && c->dim != 3) { why = "dim must be 2 or 3"; return RVE_EINVAL; }
    for (int i = 0; i < c->dim; ++i)
        if (c->n[i] < 2 || c->n[i] > 1024) { why = "n out of range [2, 1024]"; return RVE_EINVAL; }
    if (c->dim == 2 && c->n[2] != 1) { why = "n[2] must be 1 in 2D"; return RVE_EINVAL; }
    if (!(c->h > 0) || !(c->ell > 0) || !(c->k_res > 0)) { why = "h, ell, k_res must be > 0"; return RVE_EINVAL; }
    if (c->split != RVE_SPLIT_NONE) { why = "only RVE_SPLIT_NONE is available"; return RVE_EINVAL; }
    if (c->precision != RVE_PREC_FP64 && c->precision != RVE_PREC_MIXED) { why = "bad precision"; return RVE_EINVAL; }
    if (!(c->tol > 0) || !(c->tol_cg > 0) || !(c->tol_pcg > 0) || !(c->tol_al > 0)) { why = "tolerances must be > 0"; return RVE_EINVAL; }
    if (c->max_stagger < 1 || c->max_cg < 1 || c->max_pcg < 1) { why = "iteration limits must be >= 1"; return RVE_EINVAL; }
    if (c->anderson_depth < 0 || c->anderson_depth > kAndersonMax) { why = "anderson_depth in [0, 5]"; return RVE_EINVAL; }
    if (c->max_materials < 1 || c->max_materials > kMaxMat) { why = "max_materials in [1, 65536]"; return RVE_EINVAL; }
    const int s = c->dim == 2 ? 3 : 6;
    double fn = 0;
    for (int a = 0; a < s; ++a) {
        if (!std::isfinite(c->f[a])) { why = "non-finite f"; return RVE_EINVAL; }
        fn += c->f[a] * c->f[a];
    }
    if (!(fn > 0)) { why = "f must be non-zero"; return RVE_EINVAL; }
    return RVE_OK;
}

template <typename T>
static int geom_check(const rve_config* c, Geom& g, int& nbx, std::string& why) {
    AxisPlan a, b, d;
    int RB, mx, ty, my, tz, mz;
    size_t lx, ly, lz;
    if (!Solver<T>::make_geom(*c, g, a, b, d, RB, nbx, mx, lx, ty, my, ly, tz, mz, lz, why))
        return RVE_EINVAL;
    return RVE_OK;
}

extern "C" {

int rve_default_config(rve_config* c) {
    if (!c) return RVE_EINVAL;
    std::memset(c, 0, sizeof(*c));
    c->dim = 2;
    c->n[0] = c->n[1] = 64;
    c->n[2] = 1;
    c->h = 1.0;
    c->ell = 1.5;
    c->k_res = 1e-6;
    c->f[1] = 1.0;
    c->split = RVE_SPLIT_NONE;
    c->history = 1;
    c->precision = RVE_PREC_FP64;
    c->tol = 1e-8;
    c->tol_cg = 1e-10;
    c->tol_pcg = 1e-12;
    c->tol_al = 1e-10;
    c->max_stagger = 300;
    c->max_cg = 20000;
    c->max_pcg = 20000;
    c->anderson_depth = 5;
    c->frac_threshold = 0.95;
    c->A_g = 0.0;
    c->max_materials = 4096;
    return RVE_OK;
}

int rve_query_workspace(const rve_config* c, size_t* bytes) {
    std::string why;
    if (!bytes) return RVE_EINVAL;
    int rc = validate(c, why);
    if (rc) return rc;
    Geom g;
    int nbx = 1;
    Layout L;
    if (c->precision == RVE_PREC_FP64) {
        if ((rc = geom_check<double>(c, g, nbx, why))) return rc;
        Solver<double>::layout(*c, g, nbx, L, nullptr);
    } else {
        if ((rc = geom_check<float>(c, g, nbx, why))) return rc;
        Solver<float>::layout(*c, g, nbx, L, nullptr);
    }
    *bytes = L.total;
    return RVE_OK;
}

int rve_create(const rve_config* c, void* ws, size_t wsb, void* stream, rve_handle* out) {
    if (!out) return RVE_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate(c, why);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = rve_query_workspace(c, &need))) return rc;
    if (!ws) return RVE_EINVAL;
    if (wsb < need) return RVE_ENOSPC;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return RVE_EINVAL;
    auto* h = new rve_handle_s();
    h->cfg = *c;
    hipStream_t st = (hipStream_t)stream;
    if (c->precision == RVE_PREC_FP64) {
        auto* s = new Solver<double>(h, *c, ws, st);
        h->impl.reset(s);
        rc = s->init_device();
    } else {
        auto* s = new Solver<float>(h, *c, ws, st);
        h->impl.reset(s);
        rc = s->init_device();
    }
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return RVE_OK;
}

int rve_destroy(rve_handle h) {
    delete h;
    return RVE_OK;
}

int rve_set_microstructure(rve_handle h, const uint16_t* phase_id, const rve_phase* phases,
                           int nphases, const double* theta, const uint8_t* void_mask,
                           const uint8_t* phi_disc, double phi_M) {
    if (!h) return RVE_EINVAL;
    return h->impl->set_microstructure(phase_id, phases, nphases, theta, void_mask, phi_disc,
                                       phi_M);
}

int rve_step_dissipation(rve_handle h, double dtau, rve_step_info* out) {
    if (!h) return RVE_EINVAL;
    return h->impl->step(dtau, out);
}

int rve_step_dissipation_batch(rve_handle* hs, int count, const double* dtau,
                               rve_step_info* info, int* status) {
    if (!hs || count < 0 || !dtau) return RVE_EINVAL;
    std::vector<int> rcs(count, RVE_OK);
    std::vector<std::thread> th;
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) { rcs[i] = RVE_EINVAL; continue; }
        th.emplace_back([&, i]() { rcs[i] = hs[i]->impl->step(dtau[i], info ? &info[i] : nullptr); });
    }
    for (auto& t : th) t.join();
    int rc = RVE_OK;
    for (int i = 0; i < count; ++i) {
        if (status) status[i] = rcs[i];
        if (rcs[i] != RVE_OK) rc = rcs[i];
    }
    return rc;
}

int rve_effective_toughness(rve_handle h, double* G) {
    if (!h || !G) return RVE_EINVAL;
    SolverBase* s = h->impl.get();
    if (!s->ready) { h->err = "set_microstructure first"; return RVE_ESTATE; }
    if (!s->fractured) { h->err = "fracture point not reached"; return RVE_ENOTDONE; }
    *G = s->V * (s->T_c - 0.5 * s->Sigma_c * s->E_c) / s->A_g;
    return RVE_OK;
}

int rve_get_field(rve_handle h, int which, double* host, size_t count) {
    if (!h || !host) return RVE_EINVAL;
    return h->impl->get_field(which, host, count);
}

int rve_set_field(rve_handle h, int which, const double* host, size_t count) {
    if (!h || !host) return RVE_EINVAL;
    return h->impl->set_field(which, host, count);
}

int rve_get_scalars(rve_handle h, double* o) {
    if (!h || !o) return RVE_EINVAL;
    SolverBase* s = h->impl.get();
    o[0] = s->E_c;
    o[1] = s->Sigma_c;
    o[2] = s->T_c;
    o[3] = s->tau_c;
    o[4] = s->tau0;
    o[5] = s->step_c;
    return RVE_OK;
}

int rve_set_scalars(rve_handle h, const double* in) {
    if (!h || !in) return RVE_EINVAL;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(in[i])) return RVE_EINVAL;
    SolverBase* s = h->impl.get();
    s->E_c = in[0];
    s->Sigma_c = in[1];
    s->T_c = in[2];
    s->tau_c = in[3];
    s->tau0 = in[4];
    s->step_c = (int)in[5];
    return RVE_OK;
}

int rve_apply_green_op(rve_handle h, const double* eps, double* out) {
    if (!h || !eps || !out) return RVE_EINVAL;
    return h->impl->apply_green(eps, out);
}

int rve_apply_green_op_device(rve_handle h, const void* eps, void* out, int repeat) {
    if (!h || !eps || !out || repeat < 0) return RVE_EINVAL;
    return h->impl->apply_green_device(eps, out, repeat);
}

int rve_solve_mechanics(rve_handle h, int* it, double* Sigma1) {
    if (!h) return RVE_EINVAL;
    return h->impl->solve_mechanics(it, Sigma1);
}

int rve_solve_damage(rve_handle h, double E, double* D, int* it, int commit) {
    if (!h || !(E >= 0.0)) return RVE_EINVAL;
    return h->impl->solve_damage(E, D, it, commit);
}

int rve_dissipation(rve_handle h, double* D, double* G) {
    if (!h) return RVE_EINVAL;
    return h->impl->dissipation(D, G);
}

const char* rve_last_error(rve_handle h) { return h ? h->err.c_str() : "null handle"; }

const char* rve_version(void) { return "mirve 0.1 (gfx950)"; }

}  // extern "C"
