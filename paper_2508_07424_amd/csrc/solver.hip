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
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/mirve.h"
#include "kernels.h"
#include "newton.h"
#include "fft2l.h"

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

// Lattice-to-sample rotation of the z-x-z Euler angles (a1, a2, a3):
// R = R_z(a1) R_x(a2) R_z(a3); (a1, 0, 0) is the in-plane angle a1.
static void euler_rotation(double a1, double a2, double a3, double R[3][3]) {
    const double c1 = std::cos(a1), s1 = std::sin(a1), c2 = std::cos(a2), s2 = std::sin(a2);
    const double c3 = std::cos(a3), s3 = std::sin(a3);
    const double Z1[3][3] = {{c1, -s1, 0.0}, {s1, c1, 0.0}, {0.0, 0.0, 1.0}};
    const double X2[3][3] = {{1.0, 0.0, 0.0}, {0.0, c2, -s2}, {0.0, s2, c2}};
    const double Z3[3][3] = {{c3, -s3, 0.0}, {s3, c3, 0.0}, {0.0, 0.0, 1.0}};
    double T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Z1[i][k] * X2[k][j];
            T[i][j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += T[i][k] * Z3[k][j];
            R[i][j] = acc;
        }
}

// Q with mandel(R t R^T) = Q mandel(t); orthogonal.  C' = Q C Q^T.
static void mandel_rotation(const double R[3][3], double Q[6][6]) {
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
    double A[6];        // cleavage tensor, order xx, yy, zz, yz, xz, xy
};

// Cleavage tensor A_f = I + beta (I - n n) of a phase (Sec. 2.2, Eq. 15),
// n the unit lattice normal rotated by R.  2D takes its in-plane block,
// which is what projecting the rotated normal on the cross section gives
// (Sec. 5.3): a normal along z weakens every in-plane direction alike,
// A = (1 + beta) I.  With no normal (2D only), A = (1 + beta) I.
static void cleavage_tensor(const rve_phase& ph, const double R[3][3], double A[6]) {
    const double nl = std::sqrt(ph.n[0] * ph.n[0] + ph.n[1] * ph.n[1] + ph.n[2] * ph.n[2]);
    double n[3] = {0.0, 0.0, 0.0};
    if (nl > 0.0)
        for (int i = 0; i < 3; ++i)
            n[i] = (R[i][0] * ph.n[0] + R[i][1] * ph.n[1] + R[i][2] * ph.n[2]) / nl;
    const double b = ph.beta;
    A[0] = 1.0 + b * (1.0 - n[0] * n[0]);
    A[1] = 1.0 + b * (1.0 - n[1] * n[1]);
    A[2] = 1.0 + b * (1.0 - n[2] * n[2]);
    A[3] = -b * n[1] * n[2];
    A[4] = -b * n[0] * n[2];
    A[5] = -b * n[0] * n[1];
}

static HostMat phase_entry(const rve_phase& ph, const double R[3][3], bool notch, double k_res) {
    HostMat m;
    cleavage_tensor(ph, R, m.A);
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
    mandel_rotation(R, Q);
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
    pl.fastN = 0;
    int n = N, k = 0;
    while (n % 2 == 0) { n /= 2; ++k; }
    // powers of two as radix 8 and 4 (a radix 2 only for N = 2): the smallest
    // radix sets the butterflies a thread carries
    std::vector<int> r;
    int n8 = k / 3, rem = k % 3;
    if (rem == 1 && n8 > 0) { --n8; r.push_back(4); r.push_back(4); }
    else if (rem == 2) r.push_back(4);
    else if (rem == 1) r.push_back(2);
    for (int i = 0; i < n8; ++i) r.insert(r.begin(), 8);
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

// lengths served by the fixed-size two-level FFT
static bool fast_len(int N) { return N >= 16 && N <= 1024 && (N & (N - 1)) == 0; }

static int round_maxb(long long need) {
    if (need <= 1) return 1;
    if (need <= 2) return 2;
    if (need <= 4) return 4;
    if (need <= 8) return 8;
    return -1;
}

constexpr size_t kLdsCap = 60 * 1024;

// Number of Krylov iterations to enqueue before the next host check: the
// observed rate of decrease of the residual predicts how many are still
// needed, so few launches run past convergence (those exit at once).
static inline int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

struct ChunkPlanner {
    int it_prev = 0;
    double rr_prev = -1.0;
    // it: iterations done, rr: current r.r, target: r.r to reach, rr0: r.r at
    // iteration 0 (gives a rate at the first check)
    int next(int it, double rr, double target, double rr0) {
        if (rr_prev < 0.0 && rr0 > 0.0) {
            it_prev = 0;
            rr_prev = rr0;
        }
        int c = 16;
        if (rr_prev > 0.0 && it > it_prev && rr > 0.0 && rr < rr_prev && target > 0.0) {
            const double rate = std::log(rr / rr_prev) / double(it - it_prev);   // < 0
            const double need = std::log(target / rr) / rate;
            c = (int)std::ceil(need * 1.05) + 1;
        }
        it_prev = it;
        rr_prev = rr;
        return std::max(2, std::min(c, 256));
    }
};

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

// Committed host-side state of one RVE slot.
// A roctx range over a host scope: the stages of a step show up as ranges in
// a marker trace (rocprofv3 --marker-trace); without a tracer the calls do
// nothing.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

struct SlotState {
    bool ready = false;
    bool fractured = false;
    double E = 0, Sigma = 0, T = 0, tau = 0, tau0 = 0;
    double Gamma = 0;               // crack surface Gamma of the committed damage (Eq. 4)
    double V = 0, A_g = 0, min_gc = 0;
    double sig_max_prev = 0;        // max of Sigma over the committed steps before the last
    int step = 0;
};

struct SolverBase {
    virtual ~SolverBase() {}
    virtual int set_microstructure(int slot, const uint16_t*, const rve_phase*, int, const double*,
                                   const double* euler,
                                   const uint8_t*, const uint8_t*, double) = 0;
    virtual int run(const double* dtau, const int* todo, int flags, rve_step_info* info, int* status,
                    long long budget = -1) = 0;
    virtual int get_field(int slot, int which, double* host, size_t count) = 0;
    virtual int set_field(int slot, int which, const double* host, size_t count) = 0;
    virtual int apply_green(int slot, const double* eps, double* out) = 0;
    virtual int apply_green_device(const void* eps, void* out, int repeat) = 0;
    virtual int apply_green_device_scratch(void* scr, size_t cap, const void* eps, void* out,
                                           int repeat) = 0;
    virtual int solve_mechanics(int slot, int* it, double* Sigma1) = 0;
    virtual int solve_damage(int slot, double E, double* D, int* it, int commit) = 0;
    virtual int dissipation(int slot, double* D, double* G) = 0;
    virtual int profile_pass(int pass, int repeat, double* bytes_per_launch) = 0;
    virtual size_t newton_workspace(int restart) const = 0;
    // a step kept in flight by a budget run (RVE_RUN_KEEP) returns to the
    // state it began from; slot < 0: every slot
    virtual int drop_kept(int slot) = 0;
    virtual int newton_step(int slot, double dtau, const rve_newton_opts& o, void* ws, size_t ws_bytes,
                            rve_step_info* info) = 0;
    virtual int autotune(int repeat, int* shape_out) = 0;
    virtual size_t state_bytes() const = 0;
    virtual int save_state(int slot, void* host, size_t bytes) = 0;
    virtual int load_state(int slot, const void* host, size_t bytes) = 0;
    std::vector<SlotState> slots;
    int B = 1;
    // occupancy of the last rve_run_slots call: rounds (each a mechanics
    // solve, a stagger iteration or commit, one launch sequence over the
    // slots in that phase) and the slots those rounds covered in total
    long long run_rounds = 0, run_active = 0;
};

struct rve_handle_s {
    rve_config cfg;
    std::unique_ptr<SolverBase> impl;
    std::string err;
    void* scratch = nullptr;   // device address of the static scratch array on the handle's device
};

namespace mirve {

template <typename T>
struct Solver : SolverBase {
    rve_handle_s* hd;
    rve_config cfg;
    Geom g;
    AxisPlan plx, ply, plz;
    int RB = 2, nbx = 1, maxb_x = 1;
    int tly = 1, maxb_y = 1, tlz = 1, maxb_z = 1;
    // 1: the y passes of the mechanics operator stay block passes where the
    // one-wave pass (128-, 256- or 512-point y lines) applies
    int y_block = 0;
    // launch shape of the one-component passes of the damage preconditioner
    int RB1 = 2, nbx1 = 1, tly1 = 1, tlz1 = 1;
    int thr_x = 256, thr_y = 256, thr_z = 256;
    size_t lds_x = 0, lds_y = 0, lds_z = 0;
    // launch shape of the one-component passes (damage preconditioner)
    int thr_x1 = 256, thr_y1 = 256, thr_z1 = 256;
    size_t lds_x1 = 0, lds_y1 = 0, lds_z1 = 0;
    int nred = 1;
    int stream_nt = 0;               // Krylov passes stream r, p, x non-temporally
    int nmv = 1;                     // blocks per RVE of the damage direction + operator step
    hipStream_t st;
    int load_axis = 1;
    void* ws = nullptr;
    int m1_max = 1;

    // device pointers (each field holds B RVEs back to back)
    T *phi_c, *phi_w, *Hn, *psi_ini, *phi_ini, *psi1, *H, *px, *pr, *pp, *pp2, *pq, *pdinv, *pb, *tmp,
        *pz;
    T *x, *x_c, *r, *p;
    T *aF, *aG;                     // Anderson ring buffers: kHist slots of B*N
    cplx<T>* spec;
    cplx<T>* tw;
    T* dsq;                         // |d_j(k)|^2 per axis (damage preconditioner symbol)
    uint16_t* mat_id;
    MatEntry<T>* mat;
    double *partials, *cgpA, *cgpB, *cgpC, *ppA, *ppB, *sums, *dE, *dgamma;
    int *dmask[7], *dorder, *dm1, *count;
    // mixed precision: FP64 solution of the damage balance (iterative refinement)
    double* phi64 = nullptr;
    T* dlt = nullptr;                // its bulk-precision correction
    uint8_t* tmask = nullptr;       // split: tension flags of the Newton point
    T* dxs = nullptr;               // split: Newton correction (s fields)
    CgDev* cg;
    PcgDev* pcg;
    // pinned host mirrors / staging
    CgDev* h_cg = nullptr;
    PcgDev* h_pcg = nullptr;
    double* h_sums = nullptr;
    int* h_count = nullptr;
    void* h_stage = nullptr;       // ring of pinned upload slots
    size_t stage_bytes = 0;
    size_t stage_off = 0;          // next free byte; reset when the stream is drained

    int greenops = 0;
    std::vector<int> step_greens;    // Green-operator applications per slot in this step
    bool trace = false;              // MIRVE_TRACE set: stagger progress on stderr
    // captured Krylov chunks: key -> executable graph of kGraphChunk iterations
    std::map<std::string, hipGraphExec_t> graphs;
    static constexpr int kGraphChunk = 8;
    static constexpr double kGammaMax = 10.0;
    static constexpr double kFloorFactor = 10.0;
    static constexpr int kFloorWindow = 20;
    static constexpr int kMaxNewton = 100;
    std::vector<int> slope_warm;     // tmp holds a usable tangent of this slot
    // the tangent only steers Newton on E (the constraint is tested on D
    // itself): a relative error of 1e-6 in dD/dE costs nothing in the root
    static constexpr double kSlopeTol = 1e-6;
    static constexpr double kSlopeTolBulk32 = 1e-5;

    // ------------------------------------------------------------------ layout
    static long long pass_blocks_max(const Geom& g, int nbx) {
        return std::max<long long>(nbx, (g.ny * (long long)g.nz + 1) / 2);
    }
    long long pass_blocks_max() const { return pass_blocks_max(g, nbx); }
    static size_t layout(const rve_config& c, const Geom& g, int nbx, Layout& L, Solver* s) {
        const long long B = g.B;
        const size_t fN = sizeof(T) * g.N * B;
        const size_t sN = fN * g.s;
        T** single[] = {s ? &s->phi_c : nullptr, s ? &s->phi_w : nullptr, s ? &s->Hn : nullptr,
                        s ? &s->psi_ini : nullptr, s ? &s->phi_ini : nullptr, s ? &s->psi1 : nullptr,
                        s ? &s->H : nullptr, s ? &s->px : nullptr, s ? &s->pr : nullptr,
                        s ? &s->pp : nullptr, s ? &s->pp2 : nullptr, s ? &s->pq : nullptr,
                        s ? &s->pdinv : nullptr,
                        s ? &s->pb : nullptr, s ? &s->tmp : nullptr, s ? &s->pz : nullptr};
        const int ns = sizeof(single) / sizeof(single[0]);
        std::vector<size_t> offs;
        for (int i = 0; i < ns; ++i) offs.push_back(L.off(fN));
        const int m1 = std::max(0, std::min(c.anderson_depth, kAndersonMax)) + 1;
        const size_t oaF = L.off(fN * (m1 > 1 ? m1 : 1));
        const size_t oaG = L.off(fN * (m1 > 1 ? m1 : 1));
        const size_t ox = L.off(sN), oxc = L.off(sN), orr = L.off(sN), op = L.off(sN);
        const size_t ospec = L.off(sizeof(cplx<T>) * g.s * g.Nspec * B);
        const size_t otw = L.off(sizeof(cplx<T>) * (g.nx + g.ny + g.nz));
        const size_t odsq = L.off(sizeof(T) * (g.nx + g.ny + g.nz));
        const size_t omid = L.off(sizeof(uint16_t) * g.N * B);
        const size_t omat = L.off(sizeof(MatEntry<T>) * (size_t)g.mstride * B);
        const size_t opart = L.off(sizeof(double) * kMaxVals * kRedBlocks * B);
        // pass partials: one per block, sized for the smallest rows per block
        // (2), so that any launch shape the tuner picks fits
        const long long maxblk = pass_blocks_max(g, nbx);
        const size_t ocgA = L.off(sizeof(double) * maxblk * B);
        const size_t ocgB = L.off(sizeof(double) * maxblk * B);
        const size_t ocgC = L.off(sizeof(double) * maxblk * B);
        const size_t oppA = L.off(sizeof(double) * maxblk * B);
        const size_t oppB = L.off(sizeof(double) * maxblk * B);
        const size_t osums = L.off(sizeof(double) * kMaxVals * B);
        const size_t oE = L.off(sizeof(double) * B);
        const size_t ogam = L.off(sizeof(double) * kAndersonMax * B);
        size_t omask[7];
        for (int i = 0; i < 7; ++i) omask[i] = L.off(sizeof(int) * B);
        // mixed precision: the FP64 damage solution and its correction
        const bool ir = sizeof(T) < sizeof(double);
        const size_t ophi64 = ir ? L.off(sizeof(double) * g.N * B) : 0;
        const size_t odlt = ir ? L.off(fN) : 0;
        const bool split = c.split != RVE_SPLIT_NONE;
        const size_t otm = split ? L.off(sizeof(uint8_t) * g.N * B) : 0;
        const size_t odx = split ? L.off(sN) : 0;
        const size_t oord = L.off(sizeof(int) * kHist * B);
        const size_t om1 = L.off(sizeof(int) * B);
        const size_t ocnt = L.off(sizeof(int) * B);
        const size_t ocg = L.off(sizeof(CgDev) * B);
        const size_t opcg = L.off(sizeof(PcgDev) * B);
        if (s) {
            char* base = (char*)s->ws;
            for (int i = 0; i < ns; ++i) *single[i] = (T*)(base + offs[i]);
            s->aF = (T*)(base + oaF);
            s->aG = (T*)(base + oaG);
            s->x = (T*)(base + ox);
            s->x_c = (T*)(base + oxc);
            s->r = (T*)(base + orr);
            s->p = (T*)(base + op);
            s->spec = (cplx<T>*)(base + ospec);
            s->tw = (cplx<T>*)(base + otw);
            s->dsq = (T*)(base + odsq);
            s->mat_id = (uint16_t*)(base + omid);
            s->mat = (MatEntry<T>*)(base + omat);
            s->partials = (double*)(base + opart);
            s->cgpA = (double*)(base + ocgA);
            s->cgpB = (double*)(base + ocgB);
            s->cgpC = (double*)(base + ocgC);
            s->ppA = (double*)(base + oppA);
            s->ppB = (double*)(base + oppB);
            s->sums = (double*)(base + osums);
            s->dE = (double*)(base + oE);
            s->dgamma = (double*)(base + ogam);
            for (int i = 0; i < 7; ++i) s->dmask[i] = (int*)(base + omask[i]);
            s->phi64 = ir ? (double*)(base + ophi64) : nullptr;
            s->dlt = ir ? (T*)(base + odlt) : nullptr;
            s->tmask = split ? (uint8_t*)(base + otm) : nullptr;
            s->dxs = split ? (T*)(base + odx) : nullptr;
            s->dorder = (int*)(base + oord);
            s->dm1 = (int*)(base + om1);
            s->count = (int*)(base + ocnt);
            s->cg = (CgDev*)(base + ocg);
            s->pcg = (PcgDev*)(base + opcg);
        }
        return L.total;
    }

    // geometry and launch shapes from a configuration; false if unsupported
    static int threads_for(int n) { return std::min(256, ((n + 63) / 64) * 64); }
    // LDS twiddle table of a fixed-size pass: FP32 only (FP64 passes hold
    // their twiddles in registers)
    static size_t axis_tw_bytes(int N) { return sizeof(T) == 8 ? 0 : (size_t)N * sizeof(cplx<T>); }

    // Launch shape: rows per block of the x passes, lines per block of the y
    // pass, y columns per tile of the z pass (0: the default heuristic).
    struct Shape {
        int rb = 0, tly = 0, tlz = 0;
        int nt = -1;                 // streaming policy of the Krylov passes (-1: keep)
        int yblock = -1;             // 1: block y pass, 0: one-wave y pass where it applies (-1: keep)
    };

    static bool make_geom(const rve_config& c, Geom& g, AxisPlan& px, AxisPlan& py, AxisPlan& pz,
                          int& RB, int& nbx, int& maxb_x, size_t& lds_x, int& tly, int& maxb_y,
                          size_t& lds_y, int& tlz, int& maxb_z, size_t& lds_z, int& thr_x,
                          int& thr_y, int& thr_z, std::string& why, const Shape* force = nullptr) {
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
        g.B = std::max(1, c.batch);
        g.mstride = std::max(1, c.max_materials);
        g.aniso = 0;
        if (!factorize(g.nx, px) || !factorize(g.ny, py) || !factorize(g.nz, pz)) {
            why = "grid sizes must be products of 2, 3, 5, 7 (<= 1024)";
            return false;
        }
        const size_t ce = sizeof(cplx<T>);
        // x passes: RB rows per block (RB/2 packed pairs); enough blocks to fill
        // the chip (>= ~1024 over the batch), at most 16 rows
        const size_t lx = (size_t)lds_line(g.nx) * ce;
        const long long rows_total = (long long)g.ny * g.nz * g.B;
        // rows per block and lines per block are powers of two (the kernels
        // split their flat indices with shifts)
        RB = pow2_floor((int)std::max<long long>(2, std::min<long long>(16, rows_total / 1024)));
        const bool fixed = force && force->rb > 0;
        if (fixed) RB = force->rb;
        if (RB < 2 || (RB & (RB - 1))) { why = "rows per block must be a power of two >= 2"; return false; }
        // the x passes' fixed-size FFTs hold their twiddles in registers (no
        // LDS table)
        const size_t twx = 0;
        if (fast_len(g.nx)) {
            while (!fixed && RB > 2 && ((size_t)g.s * (RB / 2) * lx + twx > kLdsCap ||
                                        g.s * (RB / 2) * split_max(g.nx) > 256))
                RB /= 2;
            if ((size_t)g.s * (RB / 2) * lx + twx <= kLdsCap && g.s * (RB / 2) * split_max(g.nx) <= 256)
                px.fastN = g.nx;
        }
        auto xmb = [&](int rb) {
            return round_maxb(((long long)g.s * (rb / 2) * g.nx / px.min_rad + 255) / 256);
        };
        if (fixed && fast_len(g.nx) && !px.fastN) { why = "shape exceeds the block budget"; return false; }
        if (!px.fastN)
            while (!fixed && RB > 2 && ((size_t)g.s * (RB / 2) * lx > kLdsCap || xmb(RB) < 0)) RB /= 2;
        lds_x = (size_t)g.s * (RB / 2) * lx + (px.fastN ? twx : 0);
        maxb_x = px.fastN ? 1 : xmb(RB);
        if (lds_x > kLdsCap || maxb_x < 0) { why = "n_x too large for the LDS budget"; return false; }
        thr_x = px.fastN ? threads_for(g.s * (RB / 2) * split_max(g.nx)) : 256;
        const int nrows = g.ny * g.nz;
        nbx = (nrows + RB - 1) / RB;
        // y pass: whole contiguous lines, about 1024 elements per component per block
        auto pick = [&](AxisPlan& pl, int want, int& tl, int& mb, size_t& lds, int& thr) -> bool {
            const bool fast = fast_len(pl.N);
            for (int t = pow2_floor(std::max(1, want)); t >= 1; t /= 2) {
                const size_t l = (size_t)g.s * t * lds_line(pl.N) * ce;
                if (fast) {
                    const size_t lt = l + axis_tw_bytes(pl.N);
                    if (lt <= kLdsCap && g.s * t * split_max(pl.N) <= 256) {
                        tl = t; mb = 1; lds = lt; pl.fastN = pl.N;
                        thr = threads_for(g.s * t * split_max(pl.N));
                        return true;
                    }
                    continue;
                }
                const int m = round_maxb(((long long)g.s * t * pl.N / pl.min_rad + 255) / 256);
                if (l <= kLdsCap && m > 0) { tl = t; mb = m; lds = l; thr = 256; return true; }
            }
            return false;
        };
        // y pass: whole lines; lines per block so that the batch gives >= ~1024 blocks
        const long long ylines = (long long)g.nxh * g.nz * g.B;
        const int want_y = force && force->tly > 0
                               ? force->tly
                               : (int)std::max<long long>(1, std::min<long long>(16, ylines / 1024));
        if (!pick(py, want_y, tly, maxb_y, lds_y, thr_y)) {
            why = "n_y too large for the LDS budget";
            return false;
        }
        if (force && force->tly > 0 && tly != force->tly) { why = "y lines: a feasible power of two"; return false; }
        // z pass: a tile of y columns (up to 128 bytes per row)
        if (g.dim == 3) {
            const long long zcols = (long long)g.nxh * g.ny * g.B;
            const int want_z = force && force->tlz > 0
                                   ? force->tlz
                                   : (int)std::max<long long>(
                                         1, std::min<long long>(std::min<long long>(g.ny, 128 / ce),
                                                                zcols / 1024));
            if (!pick(pz, want_z, tlz, maxb_z, lds_z, thr_z)) {
                why = "n_z too large for the LDS budget";
                return false;
            }
            if (force && force->tlz > 0 && tlz != force->tlz) { why = "z tile: a feasible power of two"; return false; }
        }
        return true;
    }

    Solver(rve_handle_s* h, const rve_config& c, void* wsp, hipStream_t s) : hd(h), cfg(c), st(s) {
        std::string why;
        make_geom(c, g, plx, ply, plz, RB, nbx, maxb_x, lds_x, tly, maxb_y, lds_y, tlz, maxb_z,
                  lds_z, thr_x, thr_y, thr_z, why);
        ws = wsp;
        Layout L;
        layout(c, g, nbx, L, this);
        // reduction kernels: about eight voxels per thread, so that each
        // block's partial-sum reduction is amortised
        nred = (int)std::max<long long>(1, std::min<long long>((g.N + 2047) / 2048, kRedBlocks));
        // about eight voxels per thread: the per-block reduction of the
        // previous step's partials is amortised over more voxels
        nmv = (int)std::max<long long>(1, std::min<long long>(nred, (g.N + 2047) / 2048));
        // stream the Krylov vectors past the caches when r, p and x alone
        // exceed about three quarters of the 256 MB last-level cache (the
        // autotuner times both policies)
        stream_nt = 3.0 * g.s * (double)g.N * g.B * sizeof(T) > 192.0 * (1 << 20) ? 1 : 0;
        if (c.streaming >= 0) stream_nt = c.streaming;
        one_comp_shape();
        int ax = 0;
        double best = -1;
        for (int a = 0; a < g.dim; ++a)
            if (std::fabs(c.f[a]) > best) { best = std::fabs(c.f[a]); ax = a; }
        load_axis = ax;
        B = g.B;
        slots.assign(B, SlotState());
        slope_warm.assign(B, 0);
        step_greens.assign(B, 0);
        const char* tr = std::getenv("MIRVE_TRACE");
        trace = tr && *tr && *tr != '0';
        m1_max = std::max(0, std::min(c.anderson_depth, kAndersonMax)) + 1;
    }

    ~Solver() override {
        clear_graphs();
        if (h_cg) (void)hipHostFree(h_cg);
        if (h_pcg) (void)hipHostFree(h_pcg);
        if (h_sums) (void)hipHostFree(h_sums);
        if (h_count) (void)hipHostFree(h_count);
        if (h_stage) (void)hipHostFree(h_stage);
    }

    int fail(int code, const std::string& m) {
        hd->err = m;
        return code;
    }
    // a per-slot failure: status code, reason (RVE_WHY_*) and the handle's message
    std::vector<int> why_;
    void slot_fail(std::vector<int>& rcs, int b, int code, int why, const char* msg) {
        rcs[b] = code;
        if ((int)why_.size() == B) why_[b] = why;
        hd->err = std::string("slot ") + std::to_string(b) + ": " + msg;
    }

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(RVE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)
#define CHK(expr)                      \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ != RVE_OK) return rc_; \
    } while (0)

    int init_device() {
        HIPCHK(hipHostMalloc((void**)&h_cg, sizeof(CgDev) * B, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_pcg, sizeof(PcgDev) * B, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_sums, sizeof(double) * kMaxVals * B, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&h_count, sizeof(int) * B, hipHostMallocDefault));
        stage_bytes = std::max<size_t>(64 * 1024, 64 * (sizeof(double) * kHist * B + 256));
        HIPCHK(hipHostMalloc(&h_stage, stage_bytes, hipHostMallocDefault));
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
        // squared symbols of the forward differences, |d(k)|^2 = 4 sin^2(pi k / N) / h^2,
        // per axis at the same offsets
        std::vector<T> d2;
        for (int N : {g.nx, g.ny, g.nz}) {
            for (int k = 0; k < N; ++k) {
                const long double sn = std::sin(3.141592653589793238462643383279502884L * k / N);
                d2.push_back(T(4.0L * sn * sn / ((long double)g.h * g.h)));
            }
        }
        HIPCHK(hipMemcpyAsync(dsq, d2.data(), d2.size() * sizeof(T), hipMemcpyHostToDevice, st));
        // every slot starts with a valid (zero) material index and table
        HIPCHK(hipMemsetAsync(mat_id, 0, sizeof(uint16_t) * g.N * B, st));
        HIPCHK(hipMemsetAsync(mat, 0, sizeof(MatEntry<T>) * (size_t)g.mstride * B, st));
        HIPCHK(launch_fill<T>(x, T(0), g.s * g.N, B, nullptr, st));
        HIPCHK(launch_fill<T>(x_c, T(0), g.s * g.N, B, nullptr, st));
        HIPCHK(launch_fill<T>(phi_c, T(0), g.N, B, nullptr, st));
        CHK(drain());
        return RVE_OK;
    }

    int sync() {
        CHK(drain());
        return RVE_OK;
    }

    // small host -> device uploads through the pinned staging buffer
    // The copies are queued on the stream without waiting: each upload takes
    // its own slot of the pinned ring, which is only reused after the stream
    // has been drained (every drain resets the ring).
    int upload_bytes(void* dev, const void* src, size_t n) {
        const size_t need = (n + 255) & ~size_t(255);
        if (stage_off + need > stage_bytes) CHK(drain());
        char* slot = (char*)h_stage + stage_off;
        std::memcpy(slot, src, n);
        HIPCHK(hipMemcpyAsync(dev, slot, n, hipMemcpyHostToDevice, st));
        stage_off += need;
        return RVE_OK;
    }
    int upload_ints(int* dev, const std::vector<int>& v) {
        return upload_bytes(dev, v.data(), sizeof(int) * v.size());
    }
    int upload_doubles(double* dev, const std::vector<double>& v) {
        return upload_bytes(dev, v.data(), sizeof(double) * v.size());
    }
    int drain() {
        HIPCHK(hipStreamSynchronize(st));
        stage_off = 0;
        return RVE_OK;
    }
    int read_sums(int nv) {
        (void)nv;
        HIPCHK(hipMemcpyAsync(h_sums, sums, sizeof(double) * kMaxVals * B, hipMemcpyDeviceToHost, st));
        CHK(drain());
        return RVE_OK;
    }
    double sum_of(int b, int v) const { return h_sums[b * kMaxVals + v]; }

    // ---- host <-> device field copies (one slot) ---------------------------
    int upload(T* dst, const double* src, size_t n) {
        if (sizeof(T) == sizeof(double)) {
            HIPCHK(hipMemcpy(dst, src, n * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<T> tmpv(n);
            for (size_t i = 0; i < n; ++i) tmpv[i] = T(src[i]);
            HIPCHK(hipMemcpy(dst, tmpv.data(), n * sizeof(T), hipMemcpyHostToDevice));
        }
        return RVE_OK;
    }
    int download(double* dst, const T* src, size_t n) {
        CHK(drain());
        if (sizeof(T) == sizeof(double)) {
            HIPCHK(hipMemcpy(dst, src, n * sizeof(double), hipMemcpyDeviceToHost));
        } else {
            std::vector<T> tmpv(n);
            HIPCHK(hipMemcpy(tmpv.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i) dst[i] = double(tmpv[i]);
        }
        return RVE_OK;
    }

    // ---- Green operator passes --------------------------------------------
    // Mechanics CG partials: the x-forward pass of iteration k writes p.Ap
    // into pap_slot(k) (read by the x-inverse pass of k, for r, and by the
    // x-forward pass of k + 1, for x); the x-inverse pass writes r.r into
    // cgpB, read by the next x-forward pass.
    double* pap_slot(int k) const { return (k & 1) ? cgpC : cgpA; }
    // material override of the x-forward pass: ov_mat[ov_mid[i]] for every
    // slot (the Newton step's projection P = Gamma0[I:], with a table whose
    // one entry is the identity)
    const uint16_t* ov_mid = nullptr;
    const MatEntry<T>* ov_mat = nullptr;
    int fwd_x(int mode, const T* phi, const T* eps, double fcoef, double* part, const int* mask,
              int iter = 0, T* xsol = nullptr) {
        XfwdArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.pl = plx;
        a.tw = tw + plx.tw_off;
        a.mat_id = mat_id;
        a.mat = mat;
        if (ov_mat) {               // one material for every voxel (the projection)
            a.mat_id = ov_mid;
            a.mat = ov_mat;
            a.g.mstride = 0;
        }
        a.phi = phi;
        a.eps = eps;
        a.fcoef = T(fcoef);
        for (int c = 0; c < 6; ++c) a.f[c] = T(c < g.s ? cfg.f[c] : 0.0);
        a.r = r;
        a.p = p;
        a.tmask = tmask;
        a.iter = iter;
        a.active = mask;
        a.spec = spec;
        a.partials = part;
        if (mode == XF_CG || mode == XF_CG_T) {
            a.nt = stream_nt;
            a.cg = cg;
            a.x = xsol ? xsol : x;
            a.rr_part = cgpB;
            a.partials = pap_slot(iter);
            a.pap_prev = pap_slot(iter + 1);
        }
        a.rows_per_block = RB;
        a.nblocks = nbx;
        a.threads = thr_x;
        HIPCHK(launch_xfwd<T>(a, mode, maxb_x, lds_x, st));
        return RVE_OK;
    }
    dim3 grid_y(int lines) const {
        return dim3((unsigned)((g.nxh * (long long)g.nz + lines - 1) / lines), 1, B);
    }
    dim3 grid_z(int cols) const { return dim3((unsigned)(g.nxh * ((g.ny + cols - 1) / cols)), 1, B); }
    int axes(CgDev* c, const int* mask, int iter = 0) {
        AxisArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.spec = spec;
        a.cg = c;
        a.iter = iter;
        a.active = mask;
        a.pl = ply;
        a.tw = tw + ply.tw_off;
        a.contiguous = 1;
        a.lines = tly;
        a.threads = thr_y;
        a.block_only = y_block;
        if (g.dim == 2) {
            HIPCHK(launch_axis<T>(a, AX_FWD_P_INV, maxb_y, grid_y(tly), lds_y, st));
        } else {
            HIPCHK(launch_axis<T>(a, AX_FWD, maxb_y, grid_y(tly), lds_y, st));
            AxisArgs<T> bz = a;
            bz.pl = plz;
            bz.tw = tw + plz.tw_off;
            bz.contiguous = 0;
            bz.lines = tlz;
            bz.threads = thr_z;
            HIPCHK(launch_axis<T>(bz, AX_FWD_P_INV, maxb_z, grid_z(tlz), lds_z, st));
            HIPCHK(launch_axis<T>(a, AX_INV, maxb_y, grid_y(tly), lds_y, st));
        }
        return RVE_OK;
    }
    int inv_x(int mode, T* out, double scale, double* part, const int* mask, int iter = 0) {
        XinvArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.pl = plx;
        a.tw = tw + plx.tw_off;
        a.spec = spec;
        a.scale = T(scale);
        a.out = out;
        a.r = r;
        a.cg = mode == XI_CG ? cg : nullptr;
        a.nt = mode == XI_CG ? stream_nt : 0;
        a.pAp_part = pap_slot(iter);
        a.iter = iter;
        a.active = mask;
        a.partials = part;
        a.rows_per_block = RB;
        a.nblocks = nbx;
        a.threads = thr_x;
        HIPCHK(launch_xinv<T>(a, mode, maxb_x, lds_x, st));
        return RVE_OK;
    }

    // Damage preconditioner of PCG iteration k (Sec. 4.1 Eq. 24 R2 symbols):
    // after the x-forward pass applies x += alpha p, r -= alpha q (xmode
    // XF_PCG; XF_PCG0 at the start), z = S F^-1[F[S r] / (abar + bbar |d|^2)]
    // with S = sqrt(dinv).  r.r partials go to ppA, r.z partials to ppB.
    int precond_fft(int xmode, int k, T* u, const T* pdir) {
        XfwdArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.pl = plx;
        a.tw = tw + plx.tw_off;
        a.r = pr;
        a.x = u;
        a.pd = pdir;
        a.q = pq;
        a.sc = pdinv;
        a.pcg = pcg;
        a.pq_part = partials;
        a.pq_stride = (long long)kMaxVals * kRedBlocks;
        a.pq_n = nmv;
        a.iter = k;
        a.spec = spec;
        a.partials = ppA;
        a.rows_per_block = RB1;
        a.nblocks = nbx1;
        a.threads = thr_x1;
        a.nt = stream_nt;
        HIPCHK(launch_xfwd<T>(a, xmode, maxb_x, lds_x1, st));
        AxisArgs<T> y;
        std::memset(&y, 0, sizeof(y));
        y.g = g;
        y.spec = spec;
        y.pcg = pcg;
        y.iter = k;
        y.pl = ply;
        y.tw = tw + ply.tw_off;
        y.dsq = dsq;
        y.contiguous = 1;
        y.lines = tly1;
        y.threads = thr_y1;
        if (g.dim == 2) {
            HIPCHK(launch_axis<T>(y, AX_FWD_M_INV, maxb_y, grid_y(tly1), lds_y1, st));
        } else {
            HIPCHK(launch_axis<T>(y, AX_FWD, maxb_y, grid_y(tly1), lds_y1, st));
            AxisArgs<T> z = y;
            z.pl = plz;
            z.tw = tw + plz.tw_off;
            z.contiguous = 0;
            z.lines = tlz1;
            z.threads = thr_z1;
            HIPCHK(launch_axis<T>(z, AX_FWD_M_INV, maxb_z, grid_z(tlz1), lds_z1, st));
            HIPCHK(launch_axis<T>(y, AX_INV, maxb_y, grid_y(tly1), lds_y1, st));
        }
        XinvArgs<T> v;
        std::memset(&v, 0, sizeof(v));
        v.g = g;
        v.pl = plx;
        v.tw = tw + plx.tw_off;
        v.spec = spec;
        v.scale = T(1);
        v.out = pz;
        v.r = pr;
        v.sc = pdinv;
        v.pcg = pcg;
        v.iter = k;
        v.partials = ppB;
        v.rows_per_block = RB1;
        v.nblocks = nbx1;
        v.threads = thr_x1;
        v.nt = stream_nt;
        HIPCHK(launch_xinv<T>(v, XI_PCG, maxb_x, lds_x1, st));
        return RVE_OK;
    }

    // out = scale * F^-1{P : F[sigma(eps + fcoef f)]} with the handle's law
    // (g C : eps, or the volumetric split, which also records the tension
    // flags); ||out||^2 partials in part
    int green(const T* phi, const T* eps, double fcoef, T* out, double scale, double* part,
              const int* mask) {
        CHK(fwd_x(cfg.split == RVE_SPLIT_NONE ? XF_GREEN : XF_SPLIT, phi, eps, fcoef, part, mask));
        if (out == nullptr && norm_by_parseval()) {
            // only ||out||^2 is wanted: summed over the projected spectrum of
            // the forward y pass (Parseval), without the inverse transforms
            AxisArgs<T> a;
            std::memset(&a, 0, sizeof(a));
            a.g = g;
            a.pl = ply;
            a.tw = tw + ply.tw_off;
            a.spec = spec;
            a.active = mask;
            a.contiguous = 1;
            a.partials = part;
            a.nparts = nbx;
            a.nscale = scale * scale * g.inv_N;
            HIPCHK(launch_axis_norm<T>(a, st));
        } else {
            CHK(axes(nullptr, mask));
            CHK(inv_x(XI_STORE, out, scale, part, mask));
        }
        ++greenops;
        return RVE_OK;
    }
    // 2D operators with 128-, 256- or 512-point y lines take the norm of a
    // Green-operator application from its spectrum
    bool norm_by_parseval() const {
        return g.dim == 2 && g.s == 3 && (g.ny == 128 || g.ny == 256 || g.ny == 512) && ply.N == g.ny;
    }

    // masks: device int[B] built from a host vector
    int set_mask(int which, const std::vector<int>& act) { return upload_ints(dmask[which], act); }
    static bool any(const std::vector<int>& v) {
        for (int a : v)
            if (a) return true;
        return false;
    }

    // ---- (M) mechanics over the active RVEs ------------------------------------
    // CG iterations of P[C : u] = b after launch_cg_init, with the solution
    // accumulated in xsol; mode XF_CG (the law g C) or XF_CG_T (the split's
    // tangent).  Adds the iterations to iters and greens.
    void clear_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }

    // Run `enqueue(k)` for k in [k0, k0 + n): directly, or (cfg.graphs) as
    // replays of captured chunks of kGraphChunk iterations (n is rounded up;
    // iterations past a solve's end leave it unchanged).  A chunk is captured
    // once per key (the launch arguments of its iterations) and replayed.
    template <typename F>
    int run_iterations(const std::string& key, int k0, int n, F enqueue) {
        if (!cfg.graphs || st == nullptr) {     // no capture on the legacy default stream
            for (int k = k0; k < k0 + n; ++k) CHK(enqueue(k));
            return RVE_OK;
        }
        for (int c0 = k0; c0 < k0 + n; c0 += kGraphChunk) {
            const std::string gk = key + "|" + std::to_string(c0);
            auto it = graphs.find(gk);
            if (it == graphs.end()) {
                hipGraph_t gr;
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int rc = RVE_OK;
                for (int k = c0; k < c0 + kGraphChunk && rc == RVE_OK; ++k) rc = enqueue(k);
                hipError_t e = hipStreamEndCapture(st, &gr);
                CHK(rc);
                HIPCHK(e);
                hipGraphExec_t ex;
                e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                HIPCHK(e);
                it = graphs.emplace(gk, ex).first;
            }
            HIPCHK(hipGraphLaunch(it->second, st));
        }
        return RVE_OK;
    }

    int cg_loop(const T* phi, int mode, T* xsol, const std::vector<int>& act,
                std::vector<int>& iters, std::vector<int>& rcs) {
        int chunk = 8, k = 0;
        std::vector<ChunkPlanner> plan(B);
        char key[160];
        std::snprintf(key, sizeof(key), "cg:%d:%p:%p", mode, (const void*)phi, (void*)xsol);
        for (;;) {
            if (cfg.graphs && st) chunk = (chunk + kGraphChunk - 1) / kGraphChunk * kGraphChunk;
            CHK(run_iterations(key, k, chunk, [&](int kk) -> int {
                CHK(fwd_x(mode, phi, nullptr, 0.0, nullptr, nullptr, kk, xsol));
                CHK(axes(cg, nullptr, kk));
                CHK(inv_x(XI_CG, nullptr, 1.0, cgpB, nullptr, kk));
                return RVE_OK;
            }));
            k += chunk;
            HIPCHK(hipMemcpyAsync(h_cg, cg, sizeof(CgDev) * B, hipMemcpyDeviceToHost, st));
            CHK(drain());
            bool all = true;
            int next = 4;
            for (int b = 0; b < B; ++b) {
                if (!act[b] || h_cg[b].conv != kNotDone) continue;
                all = false;
                next = std::max(next, plan[b].next(k, h_cg[b].rr, h_cg[b].tol2 * h_cg[b].bn2, h_cg[b].rr0));
            }
            if (all || k > cfg.max_cg + chunk) break;
            chunk = next;
        }
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            const CgDev& c = h_cg[b];
            const int it = c.conv == kNotDone ? k : c.conv;
            iters[b] += it;
            step_greens[b] += it;
            greenops += it;
            if (c.status == 1) continue;
            if (c.status == 2) {
                if (std::isfinite(c.rr) && c.rr <= 1e4 * c.tol2 * c.bn2) continue;
                slot_fail(rcs, b, RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "mechanics CG breakdown or non-finite residual");
            } else {
                slot_fail(rcs, b, RVE_ENOCONV, RVE_WHY_CG, "mechanics CG did not converge within max_cg");
            }
        }
        return RVE_OK;
    }

    // Equilibrium for the unit load f at damage phi (Eq. 16a, Eq. 24 R1),
    // warm-started from x.
    int mech_solve(const T* phi, int mask_id, const std::vector<int>& act, std::vector<int>& iters,
                   std::vector<int>& rcs) {
        if (cfg.split != RVE_SPLIT_NONE) return mech_solve_split(phi, act, iters, rcs);
        const int* mk = dmask[mask_id];
        CHK(green(phi, nullptr, 1.0, nullptr, 1.0, cgpB, mk));          // ||b||^2
        CHK(green(phi, x, 1.0, r, -1.0, cgpA, mk));                     // r0 = -P[gC(f + x)]
        for (int b = 0; b < B; ++b)
            if (act[b]) step_greens[b] += 2;
        HIPCHK(launch_cg_init(cg, cgpA, cgpB, nbx, B, cfg.tol_cg, cfg.max_cg, mk, st));
        return cg_loop(phi, XF_CG, x, act, iters, rcs);
    }

    // With the volumetric split the law is piecewise linear: Newton steps
    // P[C_t : dx] = -P[sigma(f + x)], each by CG from dx = 0 with the tangent
    // at the tension flags of f + x, then x += dx, until
    // ||dx|| <= tol_cg ||f + x||.  Each tangent solve stops at
    // ||r|| <= tol_cg ||P[sigma(f)]|| (the load scale, as ||b|| for the
    // linear law; a tolerance relative to the shrinking Newton residual would
    // ask for accuracy below the rounding of the Green operator).
    int mech_solve_split(const T* phi, const std::vector<int>& act, std::vector<int>& iters,
                         std::vector<int>& rcs) {
        F6 f;
        for (int c = 0; c < 6; ++c) f.v[c] = c < g.s ? cfg.f[c] : 0.0;
        std::vector<int> nw(B, 0);
        for (int b = 0; b < B; ++b) nw[b] = act[b] && rcs[b] == RVE_OK;
        if (!any(nw)) return RVE_OK;
        CHK(set_mask(5, nw));
        CHK(green(phi, nullptr, 1.0, nullptr, 1.0, ppA, dmask[5]));   // ||P sigma(f)||^2 partials
        for (int b = 0; b < B; ++b)
            if (nw[b]) step_greens[b] += 1;
        for (int nt = 0; nt < kMaxNewton && any(nw); ++nt) {
            CHK(set_mask(5, nw));
            const int* mk = dmask[5];
            CHK(green(phi, x, 1.0, r, -1.0, cgpA, mk));                 // R and the flags
            for (int b = 0; b < B; ++b)
                if (nw[b]) step_greens[b] += 1;
            HIPCHK(launch_fill<T>(dxs, T(0), g.s * g.N, B, mk, st));
            HIPCHK(launch_cg_init(cg, cgpA, ppA, nbx, B, cfg.tol_cg, cfg.max_cg, mk, st));
            CHK(cg_loop(phi, XF_CG_T, dxs, nw, iters, rcs));
            HIPCHK(launch_newton_update<T>(g, x, dxs, f, partials, nred, mk, st));
            HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, mk, st));
            CHK(read_sums(2));
            for (int b = 0; b < B; ++b) {
                if (!nw[b]) continue;
                if (rcs[b] != RVE_OK) { nw[b] = 0; continue; }
                if (std::sqrt(sum_of(b, 0)) <= cfg.tol_cg * std::max(std::sqrt(sum_of(b, 1)), 1e-300))
                    nw[b] = 0;
            }
        }
        for (int b = 0; b < B; ++b)
            if (nw[b]) slot_fail(rcs, b, RVE_ENOCONV, RVE_WHY_SPLIT, "split mechanics: Newton did not converge");
        return RVE_OK;
    }

    int unit_response(const T* phi, int mask_id, T* eps1 = nullptr, T* sig1 = nullptr) {
        F6 f;
        for (int c = 0; c < 6; ++c) f.v[c] = c < g.s ? cfg.f[c] : 0.0;
        HIPCHK(launch_unit_response<T>(g, mat_id, mat, phi, x, f, cfg.split != RVE_SPLIT_NONE ? 1 : 0,
                                       psi1, eps1, sig1, partials, nred, dmask[mask_id], st));
        HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, dmask[mask_id], st));
        return read_sums(2);
    }

    // ---- (A) damage PCG over the active RVEs -----------------------------------
    // Solve a(x) u + D^T(w D u) = b (mode 0: a = Gc/l + 2 Hc, w = Gc l; mode 1:
    // a = 1, w = c) from the initial guess in u.
    int pcg_solve(const T* Hc, int mode, double c, const T* bvec, T* u, double tol, int max_it,
                  int mask_id, const std::vector<int>& act, std::vector<int>& iters,
                  std::vector<int>& rcs) {
        const int* mk = dmask[mask_id];
        const bool fft = cfg.damage_precond == RVE_PRECOND_FFT;
        HIPCHK(launch_damage_diag<T>(g, mat_id, mat, Hc, mode, c, fft ? 1 : 0, pdinv, partials, nred,
                                     mk, st));
        HIPCHK(launch_pcg_matvec<T>(g, mat_id, mat, Hc, mode, c, u, pq, nullptr, nred, nullptr, mk, st));
        HIPCHK(launch_pcg_start<T>(g, bvec, pq, pdinv, pr, partials, nred, mk, st));
        HIPCHK(launch_pcg_fin_start(pcg, partials, nred, B, tol, max_it, g.inv_N, mk, st));
        // where step 1 of each iteration finds r.z and r.r
        const double *rzp, *rrp;
        long long rzs, rrs;
        int rzn, rrn;
        if (fft) {
            CHK(precond_fft(XF_PCG0, -1, u, nullptr));
            rzp = ppB; rrp = ppA; rzs = rrs = nbx1; rzn = rrn = nbx1;
        } else {
            rzp = partials + kRedBlocks;
            rrp = partials + 2 * kRedBlocks;
            rzs = rrs = (long long)kMaxVals * kRedBlocks;
            rzn = rrn = nred;
        }
        // directions alternate between pp (even iterations) and pp2 (odd)
        int chunk = fft ? 4 : 8, k = 0;
        std::vector<ChunkPlanner> plan(B);
        char key[200];
        std::snprintf(key, sizeof(key), "pcg:%d:%.17g:%d:%p:%p", mode, c, fft ? 1 : 0, (const void*)Hc,
                      (void*)u);
        for (;;) {
            if (cfg.graphs && st) chunk = (chunk + kGraphChunk - 1) / kGraphChunk * kGraphChunk;
            CHK(run_iterations(key, k, chunk, [&](int kk) -> int {
                T* pcur = (kk & 1) ? pp2 : pp;
                T* pn = (kk & 1) ? pp : pp2;
                HIPCHK(launch_pcg_matvec_dir<T>(g, mat_id, mat, Hc, mode, c, fft ? PRE_FFT : PRE_JACOBI,
                                                pr, pdinv, pz, pcur, pn, pq, rzp, rzs, rzn, rrp, rrs,
                                                rrn, partials, nmv, pcg, kk, st));
                if (fft) CHK(precond_fft(XF_PCG, kk, u, pn));
                else HIPCHK(launch_pcg_update<T>(g, pcg, u, pr, pn, pq, pdinv, partials, nmv, nred,
                                                 kk, st));
                return RVE_OK;
            }));
            k += chunk;
            HIPCHK(hipMemcpyAsync(h_pcg, pcg, sizeof(PcgDev) * B, hipMemcpyDeviceToHost, st));
            CHK(drain());
            bool all = true;
            int next = 2;
            for (int b = 0; b < B; ++b) {
                if (!act[b] || h_pcg[b].conv != kNotDone) continue;
                all = false;
                next = std::max(next, plan[b].next(k, h_pcg[b].rr, h_pcg[b].tol2 * h_pcg[b].bn2, h_pcg[b].rr0));
            }
            if (all || k > max_it + chunk) break;
            chunk = next;
        }
        // a zero right-hand side has the solution 0 (A is positive definite);
        // the iteration stops at once for it and the warm start is cleared here
        std::vector<int> zero(B, 0);
        bool any_zero = false;
        for (int b = 0; b < B; ++b)
            if (act[b] && h_pcg[b].bn2 == 0.0) { zero[b] = 1; any_zero = true; }
        if (any_zero) {
            CHK(set_mask(4, zero));
            HIPCHK(launch_fill<T>(u, T(0), g.N, B, dmask[4], st));
        }
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            const PcgDev& d = h_pcg[b];
            iters[b] += d.conv == kNotDone ? k : d.conv;
            if (d.status == 1) continue;
            if (d.status == 2) {
                if (std::isfinite(d.rr) && (d.rr <= 1e4 * d.tol2 * d.bn2 || d.bn2 == 0.0)) continue;
                slot_fail(rcs, b, RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "damage PCG breakdown or non-finite residual");
            } else {
                slot_fail(rcs, b, RVE_ENOCONV, RVE_WHY_PCG, "damage PCG did not converge within max_pcg");
            }
        }
        return RVE_OK;
    }

    int dissip(const T* phi, int mask_id) {
        HIPCHK(launch_dissipation<T>(g, mat_id, mat, phi, partials, nred, dmask[mask_id], st));
        HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, dmask[mask_id], st));
        return read_sums(2);
    }
    double hd_() const { return std::pow(g.h, g.dim); }

    // phi(E) into u (warm start in u) for the RVEs of mask_id; D out
    int damage_at(const std::vector<double>& E, T* u, int mask_id, const std::vector<int>& act,
                  std::vector<double>& D, std::vector<int>& npcg, std::vector<int>& rcs) {
        CHK(upload_doubles(dE, E));
        HIPCHK(launch_history<T>(g, psi1, psi_ini, Hn, dE, cfg.history, H, pb, dmask[mask_id], st));
        if (phi64) return damage_refined(u, mask_id, act, D, npcg, rcs);
        CHK(pcg_solve(H, 0, 0.0, pb, u, cfg.tol_pcg, cfg.max_pcg, mask_id, act, npcg, rcs));
        CHK(dissip(u, mask_id));
        for (int b = 0; b < B; ++b)
            if (act[b]) D[b] = sum_of(b, 0) * hd_();
        return RVE_OK;
    }

    // Mixed precision: the damage balance of the load in dE solved to tol_pcg
    // by iterative refinement.  The solution phi64 is FP64 and starts from
    // the warm start in phi64; each round forms the residual 2H - A phi64 in
    // FP64 (H of Eq. 38 formed in FP64 too), solves A d = r in the bulk
    // precision to kIrInner with the bulk-type H already in H, and adds d in
    // FP64.  D(phi) comes from the FP64 field; u receives it rounded to the
    // bulk type.  An FP32 solve alone stalls near 1e-7, and a D(E) that
    // noisy keeps the constraint solve and the staggered fixed point from
    // converging near unstable crack advance.
    static constexpr int kIrMax = 12;
    static constexpr double kIrInner = 1e-4;
    int damage_refined(T* u, int mask_id, const std::vector<int>& act, std::vector<double>& D,
                       std::vector<int>& npcg, std::vector<int>& rcs) {
        std::vector<int> todo(B, 0);
        for (int b = 0; b < B; ++b) todo[b] = act[b] && rcs[b] == RVE_OK;
        for (int k = 0; any(todo); ++k) {
            CHK(set_mask(6, todo));
            HIPCHK(launch_ir_residual<T>(g, mat_id, mat, psi1, psi_ini, Hn, dE, cfg.history, phi64, pb,
                                         partials, nred, dmask[6], st));
            HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, dmask[6], st));
            CHK(read_sums(2));
            std::vector<int> zero(B, 0), more(B, 0);
            for (int b = 0; b < B; ++b) {
                if (!todo[b]) continue;
                const double rr = sum_of(b, 0), bb = sum_of(b, 1);
                if (!std::isfinite(rr)) {
                    slot_fail(rcs, b, RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "non-finite damage residual");
                    todo[b] = 0;
                } else if (bb == 0.0) {
                    zero[b] = 1;            // the solution of a zero right-hand side is 0
                    todo[b] = 0;
                } else if (rr <= cfg.tol_pcg * cfg.tol_pcg * bb) {
                    todo[b] = 0;
                } else if (k >= kIrMax) {
                    slot_fail(rcs, b, RVE_ENOCONV, RVE_WHY_PCG, "damage refinement did not converge");
                    todo[b] = 0;
                } else {
                    more[b] = 1;
                }
            }
            if (any(zero)) {
                CHK(set_mask(6, zero));
                HIPCHK(launch_fill<double>(phi64, 0.0, g.N, B, dmask[6], st));
            }
            if (!any(more)) break;
            CHK(set_mask(6, more));
            HIPCHK(launch_fill<T>(dlt, T(0), g.N, B, dmask[6], st));
            CHK(pcg_solve(H, 0, 0.0, pb, dlt, kIrInner, cfg.max_pcg, 6, more, npcg, rcs));
            for (int b = 0; b < B; ++b)
                if (more[b] && rcs[b] != RVE_OK) { more[b] = 0; todo[b] = 0; }
            CHK(set_mask(6, more));
            HIPCHK(launch_ir_update<T>(phi64, dlt, (T*)nullptr, g.N, B, dmask[6], st));
        }
        const int* mk = dmask[mask_id];
        HIPCHK(launch_ir_update<T>(phi64, (const T*)nullptr, u, g.N, B, mk, st));
        HIPCHK(launch_dissipation64<T>(g, mat_id, mat, phi64, partials, nred, mk, st));
        HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, mk, st));
        CHK(read_sums(2));
        for (int b = 0; b < B; ++b)
            if (act[b]) D[b] = sum_of(b, 0) * hd_();
        return RVE_OK;
    }

    // dD/dE at (E, u = phi(E)) via the tangent system with the same H (dE holds E)
    int damage_slope(T* u, int mask_id, const std::vector<int>& act, std::vector<double>& dD,
                     std::vector<int>& npcg, std::vector<int>& rcs) {
        const int* mk = dmask[mask_id];
        HIPCHK(launch_tangent_rhs<T>(g, u, psi1, psi_ini, Hn, dE, cfg.history, pb, mk, st));
        // warm start from the slot's previous tangent (zero when it has none)
        std::vector<int> reset(B, 0);
        bool any_reset = false;
        for (int b = 0; b < B; ++b)
            if (act[b] && !slope_warm[b]) { reset[b] = 1; any_reset = true; }
        if (any_reset) {
            CHK(set_mask(4, reset));
            HIPCHK(launch_fill<T>(tmp, T(0), g.N, B, dmask[4], st));
        }
        // the tangent only steers Newton on E (the constraint is tested on D
        // itself), so it is solved to a looser tolerance
        const double tol = std::max(sizeof(T) < sizeof(double) ? kSlopeTolBulk32 : cfg.tol_pcg,
                                    kSlopeTol);
        CHK(pcg_solve(H, 0, 0.0, pb, tmp, tol, cfg.max_pcg, mask_id, act, npcg, rcs));
        for (int b = 0; b < B; ++b)
            if (act[b]) slope_warm[b] = rcs[b] == RVE_OK ? 1 : 0;
        HIPCHK(launch_dissipation_dir<T>(g, mat_id, mat, u, tmp, partials, nred, mk, st));
        HIPCHK(launch_sum_partials(partials, nred, 1, B, sums, mk, st));
        CHK(read_sums(1));
        for (int b = 0; b < B; ++b)
            if (act[b]) dD[b] = sum_of(b, 0) * hd_();
        return RVE_OK;
    }

    // E >= 0 with D(phi(E)) = tau (Eq. 16c) for every active RVE; phi(E) left in u.
    // Uses masks 2 and 3.
    int arclength(const std::vector<double>& tau, const std::vector<double>& E0, T* u,
                  const std::vector<int>& act, std::vector<double>& Eout, std::vector<int>& npcg,
                  std::vector<int>& rcs) {
        std::vector<double> lo(B, 0.0), hi(B, INFINITY), E(B, 0.0), D(B, 0.0), dD(B, 0.0);
        std::vector<int> al(B, 0);
        bool need_guess = false;
        for (int b = 0; b < B; ++b) {
            al[b] = act[b] && rcs[b] == RVE_OK;
            E[b] = E0[b];
            if (al[b] && !(E[b] > 0.0)) need_guess = true;
        }
        if (need_guess) {
            CHK(set_mask(2, al));
            HIPCHK(launch_max_field<T>(psi1, g.N, B, partials, nred, dmask[2], st));
            HIPCHK(launch_max_partials(partials, nred, B, sums, dmask[2], st));
            CHK(read_sums(1));
            for (int b = 0; b < B; ++b) {
                if (!al[b] || E[b] > 0.0) continue;
                const double pm = sum_of(b, 0);
                E[b] = pm > 0.0 ? std::sqrt(slots[b].min_gc / cfg.ell / pm) : 1.0;
            }
        }
        for (int it = 0; it < 200 && any(al); ++it) {
            CHK(set_mask(2, al));
            CHK(damage_at(E, u, 2, al, D, npcg, rcs));
            std::vector<int> sl(B, 0);
            for (int b = 0; b < B; ++b) {
                if (!al[b]) continue;
                if (rcs[b] != RVE_OK) { al[b] = 0; continue; }
                if (std::fabs(D[b] - tau[b]) <= cfg.tol_al * tau[b]) {
                    Eout[b] = E[b];
                    al[b] = 0;
                    continue;
                }
                if (D[b] < tau[b]) lo[b] = std::max(lo[b], E[b]);
                else hi[b] = std::min(hi[b], E[b]);
                // a bracket narrower than the resolution of D(E) ends the search
                const double res = sizeof(T) == sizeof(double) ? 1e-15 : 1e-9;
                if (!std::isinf(hi[b]) && hi[b] - lo[b] <= res * hi[b]) {
                    Eout[b] = E[b];
                    al[b] = 0;
                    continue;
                }
                sl[b] = 1;
            }
            if (!any(sl)) continue;
            CHK(set_mask(3, sl));
            CHK(damage_slope(u, 3, sl, dD, npcg, rcs));
            for (int b = 0; b < B; ++b) {
                if (!sl[b]) continue;
                if (rcs[b] != RVE_OK) { al[b] = 0; continue; }
                double En = dD[b] > 0.0 ? E[b] - (D[b] - tau[b]) / dD[b] : NAN;
                if (!(lo[b] < En && En < hi[b]))
                    En = std::isinf(hi[b]) ? 2.0 * E[b] : 0.5 * (lo[b] + hi[b]);
                E[b] = En;
            }
        }
        for (int b = 0; b < B; ++b)
            if (al[b] && rcs[b] == RVE_OK)
                slot_fail(rcs, b, RVE_ENOCONV, RVE_WHY_ARCLENGTH, "dissipation constraint (arc-length) did not converge");
        return RVE_OK;
    }

    // ---- Anderson mixing (host side of the small least-squares problems) ------
    int anderson_mix(const std::vector<int>& mixing, const std::vector<int>& nhist, T* out,
                     std::vector<int>& rcs) {
        std::vector<int> order(kHist * B, 0), m1(B, 1);
        for (int b = 0; b < B; ++b) {
            if (!mixing[b]) continue;
            m1[b] = std::min(nhist[b], m1_max);
            for (int i = 0; i < m1[b]; ++i) order[b * kHist + i] = (nhist[b] - m1[b] + i) % m1_max;
        }
        CHK(upload_ints(dorder, order));
        CHK(upload_ints(dm1, m1));
        CHK(set_mask(3, mixing));
        const long long sstride = g.N * (long long)B;
        // about 16 voxels per thread: the block reduction of the 30 Gram
        // entries is amortised over more voxels
        const int ngr = (int)std::max<long long>(1, std::min<long long>(nred, (g.N + 4095) / 4096));
        HIPCHK(launch_anderson_gram<T>(g, aF, sstride, dorder, dm1, partials, ngr, dmask[3], st));
        const int nv = kAndersonMax * kAndersonMax + kAndersonMax;
        HIPCHK(launch_sum_partials(partials, ngr, nv, B, sums, dmask[3], st));
        CHK(read_sums(nv));
        std::vector<double> gam(kAndersonMax * B, 0.0);
        for (int b = 0; b < B; ++b) {
            if (!mixing[b]) continue;
            const int m = m1[b] - 1;
            const double* hs = h_sums + b * kMaxVals;
            // normal equations (dF^T dF + ridge) gamma = dF^T F_m
            double A[kAndersonMax][kAndersonMax], bv[kAndersonMax];
            double tr = 0.0;
            for (int a = 0; a < m; ++a) tr += hs[a * kAndersonMax + a];
            // FP32 fields carry noise of about 1e-7 in the residual differences:
            // the ridge keeps the small least-squares problem above it
            const double ridge = sizeof(T) == sizeof(double) ? 1e-14 : 1e-6;
            for (int a = 0; a < m; ++a) {
                for (int c = 0; c < m; ++c) A[a][c] = hs[a * kAndersonMax + c];
                A[a][a] += ridge * tr;
                bv[a] = hs[kAndersonMax * kAndersonMax + a];
            }
            bool ok = true;
            for (int k = 0; k < m && ok; ++k) {
                int piv = k;
                for (int i = k + 1; i < m; ++i)
                    if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
                if (piv != k) {
                    for (int j = 0; j < m; ++j) std::swap(A[k][j], A[piv][j]);
                    std::swap(bv[k], bv[piv]);
                }
                if (A[k][k] == 0.0) { ok = false; break; }
                for (int i = k + 1; i < m; ++i) {
                    const double f = A[i][k] / A[k][k];
                    for (int j = k; j < m; ++j) A[i][j] -= f * A[k][j];
                    bv[i] -= f * bv[k];
                }
            }
            double* gb = &gam[b * kAndersonMax];
            for (int k = m - 1; k >= 0 && ok; --k) {
                double s = bv[k];
                for (int j = k + 1; j < m; ++j) s -= A[k][j] * gb[j];
                gb[k] = s / A[k][k];
            }
            double gsum = 0.0;
            for (int k = 0; k < m; ++k) {
                if (!std::isfinite(gb[k])) ok = false;
                gsum += std::fabs(gb[k]);
            }
            // FP32: an extrapolation far outside the history is noise; take the
            // plain fixed-point step instead (gamma = 0 gives phi(E))
            if (ok && sizeof(T) != sizeof(double) && gsum > kGammaMax)
                for (int k = 0; k < m; ++k) gb[k] = 0.0;
            if (!ok) slot_fail(rcs, b, RVE_ENUMERIC, RVE_WHY_ANDERSON, "singular or non-finite Anderson system");
        }
        CHK(upload_doubles(dgamma, gam));
        HIPCHK(launch_anderson_mix<T>(g, aG, sstride, dorder, dm1, dgamma, out, dmask[3], st));
        return RVE_OK;
    }

    // ---- microstructure of one slot ---------------------------------------------
    // Orientations: theta[N] (about z), or euler[3 N] (z-x-z angles per voxel).
    int set_microstructure(int slot, const uint16_t* pid, const rve_phase* phases, int nph,
                           const double* theta, const double* euler, const uint8_t* vmask,
                           const uint8_t* disc, double phi_M) override {
        Range rg("mirve: microstructure + enrichment (Eq. 35-38)");
        if (slot < 0 || slot >= B) return fail(RVE_EINVAL, "slot out of range");
        CHK(drop_kept(slot));
        if (!pid || !phases || nph <= 0) return fail(RVE_EINVAL, "phase_id and phases required");
        if (!(phi_M > 0.0 && phi_M < 1.0)) return fail(RVE_EINVAL, "phi_M must be in (0, 1)");
        for (int i = 0; i < nph; ++i) {
            const rve_phase& ph = phases[i];
            if (!(ph.Gc > 0.0) || !std::isfinite(ph.Gc)) return fail(RVE_EINVAL, "Gc must be > 0");
            if (!std::isfinite(ph.beta) || !(ph.beta > -1.0))
                return fail(RVE_EINVAL, "cleavage weight beta must be finite and > -1");
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(ph.n[a])) return fail(RVE_EINVAL, "non-finite cleavage normal");
            if (ph.beta != 0.0 && g.dim == 3 && ph.n[0] == 0.0 && ph.n[1] == 0.0 && ph.n[2] == 0.0)
                return fail(RVE_EINVAL, "a phase with beta != 0 needs a cleavage normal n");
            if (ph.kind == RVE_PHASE_ISO) {
                if (!(ph.E > 0.0) || !std::isfinite(ph.E) || !(ph.nu > -1.0 && ph.nu < 0.5))
                    return fail(RVE_EINVAL, "isotropic phase needs E > 0, -1 < nu < 0.5");
            } else if (ph.kind == RVE_PHASE_CUBIC) {
                if (!std::isfinite(ph.C11) || !std::isfinite(ph.C12) || !std::isfinite(ph.C44) ||
                    !(ph.C11 > std::fabs(ph.C12)) || !(ph.C11 + 2 * ph.C12 > 0) || !(ph.C44 > 0))
                    return fail(RVE_EINVAL, "cubic phase is not positive definite");
            } else {
                return fail(RVE_EINVAL, "unknown phase kind");
            }
        }
        // every input is checked (and the material table built) before the
        // slot is touched
        if (theta && euler) return fail(RVE_EINVAL, "theta and euler are exclusive");
        std::map<std::tuple<int, double, double, double, int>, int> keys;
        std::vector<uint16_t> ids(g.N);
        std::vector<MatEntry<T>> table;
        double min_gc = INFINITY;
        for (long long i = 0; i < g.N; ++i) {
            const int ph = pid[i];
            if (ph >= nph) return fail(RVE_EINVAL, "phase_id out of range");
            double ang[3] = {theta ? theta[i] : 0.0, 0.0, 0.0};
            if (euler)
                for (int a = 0; a < 3; ++a) ang[a] = euler[3 * i + a];
            if (!std::isfinite(ang[0]) || !std::isfinite(ang[1]) || !std::isfinite(ang[2]))
                return fail(RVE_EINVAL, "non-finite orientation angle");
            const int nt = vmask ? (vmask[i] ? 1 : 0) : 0;
            // the angles matter for rotated stiffness and for cleavage tensors
            const bool by_angle = phases[ph].kind != RVE_PHASE_ISO || phases[ph].beta != 0.0;
            if (!by_angle) ang[0] = ang[1] = ang[2] = 0.0;
            auto key = std::make_tuple(ph, ang[0], ang[1], ang[2], nt);
            auto it = keys.find(key);
            int id;
            if (it == keys.end()) {
                id = (int)table.size();
                if (id >= g.mstride || id >= kMaxMat)
                    return fail(RVE_EINVAL, "more distinct materials than max_materials");
                keys[key] = id;
                double R[3][3];
                euler_rotation(ang[0], ang[1], ang[2], R);
                HostMat hm = phase_entry(phases[ph], R, nt != 0, cfg.k_res);
                MatEntry<T> me;
                std::memset(&me, 0, sizeof(me));
                static const int in2d[3] = {0, 1, 5};
                for (int a = 0; a < g.s; ++a)
                    for (int c = 0; c < g.s; ++c) {
                        const int ia = g.dim == 2 ? in2d[a] : a;
                        const int ic = g.dim == 2 ? in2d[c] : c;
                        me.C[a * g.s + c] = T(hm.C[ia][ic]);
                    }
                me.K = T(hm.K);
                me.Gc = T(hm.Gc);
                me.drive = T(hm.drive);
                for (int a = 0; a < 6; ++a) me.A[a] = T(hm.A[a]);
                table.push_back(me);
            } else {
                id = it->second;
            }
            ids[i] = (uint16_t)id;
            min_gc = std::min(min_gc, phases[ph].Gc);
        }
        slope_warm[slot] = 0;
        // a handle whose slots have a cleavage tensor switches its damage
        // kernels to the anisotropic stencil (graphs captured before hold the
        // isotropic one)
        bool aniso = false;
        for (int i = 0; i < nph; ++i) aniso = aniso || phases[i].beta != 0.0;
        if (aniso && !g.aniso) {
            g.aniso = 1;
            clear_graphs();
        }
        SlotState& S = slots[slot];
        S.ready = false;
        S.min_gc = min_gc;
        CHK(drain());
        HIPCHK(hipMemcpy(mat_id + (long long)slot * g.N, ids.data(), sizeof(uint16_t) * g.N,
                         hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(mat + (long long)slot * g.mstride, table.data(),
                         sizeof(MatEntry<T>) * table.size(), hipMemcpyHostToDevice));
        // reference crack area: lines along the load axis without a notch voxel
        if (cfg.A_g > 0) {
            S.A_g = cfg.A_g;
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
            S.A_g = double(lines) * std::pow(g.h, g.dim - 1);
        }
        S.V = double(g.N) * hd_();
        std::vector<int> one(B, 0);
        one[slot] = 1;
        CHK(set_mask(0, one));
        const int* mk = dmask[0];
        const long long so = (long long)slot * g.N;
        // crack-tip enrichment (Eq. 35): (1 + l^2 D^T D) phi_o = phi_disc
        bool anyd = false;
        std::vector<double> d(g.N, 0.0);
        if (disc)
            for (long long i = 0; i < g.N; ++i)
                if (disc[i]) { d[i] = 1.0; anyd = true; }
        HIPCHK(launch_fill<T>(phi_ini, T(0), g.N, B, mk, st));
        if (anyd) {
            CHK(upload(pb + so, d.data(), g.N));
            std::vector<int> it(B, 0), rcs(B, RVE_OK);
            const double ctol = sizeof(T) == 8 ? 1e-15 : 1e-7;
            CHK(pcg_solve(nullptr, 1, cfg.ell * cfg.ell, pb, phi_ini, ctol, 100000, 0, one, it, rcs));
            if (rcs[slot] != RVE_OK) return rcs[slot];
            HIPCHK(launch_max_field<T>(phi_ini, g.N, B, partials, nred, mk, st));
            HIPCHK(launch_max_partials(partials, nred, B, sums, mk, st));
            HIPCHK(launch_scale_field<T>(phi_ini, sums, phi_M, g.N, B, mk, st));
        }
        HIPCHK(launch_psi_ini<T>(g, mat_id, mat, phi_ini, psi_ini, mk, st));
        HIPCHK(launch_copy<T>(phi_ini, phi_c, g.N, B, mk, st));
        HIPCHK(launch_copy<T>(psi_ini, Hn, g.N, B, mk, st));
        HIPCHK(launch_fill<T>(x, T(0), g.s * g.N, B, mk, st));
        HIPCHK(launch_fill<T>(x_c, T(0), g.s * g.N, B, mk, st));
        HIPCHK(launch_fill<T>(psi1, T(0), g.N, B, mk, st));
        CHK(dissip(phi_c, 0));
        S.tau = S.tau0 = sum_of(slot, 0) * hd_();
        S.Gamma = sum_of(slot, 1) * hd_();
        if (!std::isfinite(S.tau)) return fail(RVE_ENUMERIC, "non-finite initial dissipation");
        S.E = S.Sigma = S.T = 0.0;
        S.sig_max_prev = 0.0;
        S.step = 0;
        S.fractured = false;
        S.ready = true;
        return RVE_OK;
    }

    // ---- dissipation-controlled steps, every slot at its own pace ---------------
    // Progress of one slot during an rve_run_slots call.  A step of dtau is an
    // attempt at the full increment; an attempt that fails (any solver limit
    // or a breakdown) leaves the committed state unchanged and is replaced by
    // two attempts of half the increment, recursively down to max_halvings
    // (dissipation control allows any subdivision of the increment).  If the
    // deepest attempt fails too, the slot returns to the state it had when
    // the step began.
    struct Progress {
        int stage = 0;                 // 0 nothing to do, 1 stagger, 2 final equilibrium + commit
        int todo = 0;                  // steps still to take
        double dtau = 0.0;             // increment of a step
        std::deque<std::pair<double, int>> pend;   // sub-steps of the step: (increment, depth)
        double tau = 0.0, E = 0.0;     // target dissipation and load of the attempt
        int it = 0, nhist = 0;         // stagger iterations and Anderson history of the attempt
        double ref = INFINITY;         // stall detection: best error, halved at iteration ref_it
        int ref_it = 0;
        bool sub_done = false;         // a sub-step of the step has been committed
        bool snap = false;             // s_* hold the state at the start of the step
        std::vector<char> s_phi, s_H, s_x, s_tan;
        SlotState s_state;
        int s_warm = 0;
        bool stop_frac = false;
        int n_steps = 0, n_sub = 0, n_stag = 0, n_cg = 0, n_pcg = 0, n_green = 0;
        int status = RVE_OK, reason = RVE_WHY_NONE;
        bool has_last = false;
        rve_step_info last{};
        bool pre_has_last = false;     // last / has_last as the current step began
        rve_step_info pre_last{};
        int pre_sub = 0, pre_stag = 0, pre_cg = 0, pre_pcg = 0, pre_green = 0;   // counters then
        bool recount = false;          // take pre_* again once the round's work is counted
    };

    void begin_step(Progress& q) {
        q.pend.clear();
        q.pend.push_back({q.dtau, 0});
        q.sub_done = false;
        q.pre_has_last = q.has_last;
        q.pre_last = q.last;
        mark_counters(q);
        q.snap = false;
        q.s_phi.clear(); q.s_H.clear(); q.s_x.clear(); q.s_tan.clear();
    }
    static void mark_counters(Progress& q) {
        q.pre_sub = q.n_sub; q.pre_stag = q.n_stag; q.pre_cg = q.n_cg;
        q.pre_pcg = q.n_pcg; q.pre_green = q.n_green;
        q.recount = false;
    }
    void begin_attempt(int b, Progress& q, std::vector<int>& fresh) {
        q.tau = slots[b].tau + q.pend.front().first;
        q.E = slots[b].E;
        q.it = 0;
        q.nhist = 0;
        q.ref = INFINITY;
        q.ref_it = 0;
        q.stage = 1;
        fresh[b] = 1;                  // phi_w <- phi_c, x <- x_c before the next equilibrium
    }

    // host copies of the committed fields of one slot (raw bytes of the bulk type)
    int save_fields(int b, std::vector<char>& sphi, std::vector<char>& sH, std::vector<char>& sx,
                    std::vector<char>& stan) {
        CHK(drain());
        const size_t fN = sizeof(T) * g.N, sN = fN * g.s;
        sphi.resize(fN); sH.resize(fN); sx.resize(sN); stan.resize(fN);
        HIPCHK(hipMemcpy(sphi.data(), phi_c + (long long)b * g.N, fN, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(sH.data(), Hn + (long long)b * g.N, fN, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(sx.data(), x_c + (long long)b * g.s * g.N, sN, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(stan.data(), tmp + (long long)b * g.N, fN, hipMemcpyDeviceToHost));
        return RVE_OK;
    }
    int load_fields(int b, const char* sphi, const char* sH, const char* sx, const char* stan) {
        CHK(drain());
        const size_t fN = sizeof(T) * g.N, sN = fN * g.s;
        HIPCHK(hipMemcpy(phi_c + (long long)b * g.N, sphi, fN, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(Hn + (long long)b * g.N, sH, fN, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(x_c + (long long)b * g.s * g.N, sx, sN, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(x + (long long)b * g.s * g.N, sx, sN, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(tmp + (long long)b * g.N, stan, fN, hipMemcpyHostToDevice));
        return RVE_OK;
    }

    // Slot b stops in the middle of a step (a step budget was reached): the
    // step does not happen; sub-steps of it that had committed are undone,
    // and the work counters drop the step's work.
    int abandon_step(int b, Progress& q) {
        if (q.stage == 0) return RVE_OK;
        q.n_sub = q.pre_sub; q.n_stag = q.pre_stag; q.n_cg = q.pre_cg;
        q.n_pcg = q.pre_pcg; q.n_green = q.pre_green;
        if (q.sub_done) {
            if (!q.snap) return fail(RVE_EDEVICE, "no snapshot of the step's start");
            CHK(load_fields(b, q.s_phi.data(), q.s_H.data(), q.s_x.data(), q.s_tan.data()));
            slots[b] = q.s_state;
            slope_warm[b] = q.s_warm;
            q.has_last = q.pre_has_last;
            q.last = q.pre_last;
        } else {
            // the working fields are copies; only the strain warm start moved
            const long long so = (long long)b * g.s * g.N;
            HIPCHK(hipMemcpyAsync(x + so, x_c + so, sizeof(T) * g.s * g.N, hipMemcpyDeviceToDevice, st));
        }
        q.stage = 0;
        q.todo = 0;
        return RVE_OK;
    }

    // Steps kept in flight between budget runs (RVE_RUN_KEEP): the slot's
    // progress, with its working damage, strain and Anderson history left on
    // the device.  Every other call that reads or changes a slot drops its
    // kept step first.
    std::vector<Progress> kept;
    int drop_kept(int slot) override {
        if (kept.empty()) return RVE_OK;
        for (int b = 0; b < B; ++b) {
            if ((slot >= 0 && b != slot) || kept[b].stage == 0) continue;
            CHK(abandon_step(b, kept[b]));
            kept[b] = Progress();
        }
        return RVE_OK;
    }

    // A failed attempt of slot b (its working strain is already reset).
    int on_failure(int b, Progress& q, int code, int why, std::vector<int>& fresh) {
        const auto cur = q.pend.front();
        const bool retry = (code == RVE_ENOCONV || code == RVE_ENUMERIC) && cur.second < cfg.max_halvings;
        if (retry) {
            // the first failure of a step comes before any of its sub-steps has
            // committed: the committed state is still the one the step began from
            if (!q.snap) {
                CHK(save_fields(b, q.s_phi, q.s_H, q.s_x, q.s_tan));
                q.s_state = slots[b];
                q.s_warm = slope_warm[b];
                q.snap = true;
            }
            q.pend.pop_front();
            q.pend.push_front({0.5 * cur.first, cur.second + 1});
            q.pend.push_front({0.5 * cur.first, cur.second + 1});
            begin_attempt(b, q, fresh);
            return RVE_OK;
        }
        if (q.sub_done) {              // transactional: back to the start of the step
            CHK(load_fields(b, q.s_phi.data(), q.s_H.data(), q.s_x.data(), q.s_tan.data()));
            slots[b] = q.s_state;
            slope_warm[b] = q.s_warm;
            q.has_last = q.pre_has_last;
            q.last = q.pre_last;
        }
        q.status = code;
        q.reason = why;
        q.stage = 0;
        q.todo = 0;
        return RVE_OK;
    }

    // Slots b with todo[b] > 0 take up to todo[b] steps of dtau[b] each
    // (Eq. 16), at their own pace: a slot that commits a step starts its next
    // one in the following round, while other slots are still iterating.
    // Every launch of a round covers the slots that are in that phase.
    // budget >= 0: the call ends once the slots together have committed that
    // many steps (at the end of the round in which it is reached); a slot
    // then in the middle of a step returns to the state the step began from.
    int run(const double* dtau, const int* todo, int flags, rve_step_info* info, int* status,
            long long budget = -1) override {
        Range rg("mirve: rve_run_slots");
        std::vector<Progress> P(B);
        std::vector<int> fresh(B, 0);
        const bool keep = (flags & RVE_RUN_KEEP) && budget >= 0;
        if (kept.empty()) kept.resize(B);
        std::vector<int> resume(B, 0);
        for (int b = 0; b < B; ++b) {
            if (kept[b].stage == 0) continue;
            const bool sf = (flags & RVE_RUN_STOP_AT_FRACTURE) != 0;
            resume[b] = keep && todo[b] > 0 && dtau[b] == kept[b].dtau && slots[b].ready &&
                        !(sf && slots[b].fractured);
            if (!resume[b]) CHK(drop_kept(b));
        }
        for (int b = 0; b < B; ++b) {
            Progress& q = P[b];
            if (resume[b]) {
                // the kept step goes on from where the last call left it; this
                // call's counters start at zero.  An attempt that had not run
                // a round yet still takes its fresh working fields.
                q = std::move(kept[b]);
                kept[b] = Progress();
                if (q.stage == 1 && q.it == 0) fresh[b] = 1;
                q.todo = todo[b];
                q.stop_frac = (flags & RVE_RUN_STOP_AT_FRACTURE) != 0;
                q.n_steps = q.n_sub = q.n_stag = q.n_cg = q.n_pcg = q.n_green = 0;
                mark_counters(q);
                q.has_last = q.pre_has_last = false;
                q.status = RVE_OK;
                q.reason = RVE_WHY_NONE;
                continue;
            }
            if (todo[b] <= 0 || dtau[b] == 0.0) continue;
            if (!slots[b].ready) { q.status = RVE_ESTATE; hd->err = "set_microstructure first"; continue; }
            if (!(dtau[b] > 0.0) || !std::isfinite(dtau[b])) {
                q.status = RVE_EINVAL;
                hd->err = "dtau must be finite and > 0";
                continue;
            }
            q.stop_frac = (flags & RVE_RUN_STOP_AT_FRACTURE) != 0;
            if (q.stop_frac && slots[b].fractured) continue;
            q.todo = todo[b];
            q.dtau = dtau[b];
            begin_step(q);
            begin_attempt(b, q, fresh);
        }
        run_rounds = run_active = 0;
        for (;;) {
            if (budget >= 0) {
                long long done = 0;
                for (int b = 0; b < B; ++b) done += P[b].n_steps;
                if (done >= budget) {
                    for (int b = 0; b < B; ++b) {
                        if (keep && P[b].stage != 0) kept[b] = P[b];
                        else CHK(abandon_step(b, P[b]));
                    }
                    break;
                }
            }
            std::vector<int> M(B, 0);
            for (int b = 0; b < B; ++b) M[b] = P[b].stage != 0;
            if (!any(M)) break;
            run_rounds += 1;
            for (int b = 0; b < B; ++b) run_active += M[b];
            if (any(fresh)) {
                CHK(set_mask(0, fresh));
                HIPCHK(launch_copy<T>(phi_c, phi_w, g.N, B, dmask[0], st));
                HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, B, dmask[0], st));
                fresh.assign(B, 0);
            }
            std::vector<int> rc(B, RVE_OK), ncg(B, 0), npcg(B, 0);
            why_.assign(B, RVE_WHY_NONE);
            step_greens.assign(B, 0);
            // (M) equilibrium at the working damage of every slot of the round
            CHK(set_mask(1, M));
            {
                Range rg("mirve: equilibrium (Eq. 16a)");
                CHK(mech_solve(phi_w, 1, M, ncg, rc));
            }
            std::vector<int> ok(B, 0), C(B, 0), S(B, 0);
            for (int b = 0; b < B; ++b) ok[b] = M[b] && rc[b] == RVE_OK;
            std::vector<double> S1(B, 0.0), s2(B, 0.0);
            if (any(ok)) {
                CHK(set_mask(1, ok));
                CHK(unit_response(phi_w, 1));
                for (int b = 0; b < B; ++b) {
                    if (!ok[b]) continue;
                    S1[b] = sum_of(b, 0) / double(g.N);
                    s2[b] = sum_of(b, 1);
                    (P[b].stage == 2 ? C : S)[b] = 1;
                }
            }
            // (A), (U) one stagger iteration of the slots still iterating; the
            // slots committing below start their next attempt in the next round
            if (any(S)) {
                Range rg("mirve: constraint + damage (Eq. 16b, 16c)");
                CHK(stagger_iteration(S, P, rc, npcg));
            }
            if (any(C)) {
                Range rg("mirve: commit (Eq. 33, 38)");
                CHK(commit(C, S1, s2, P, fresh));
            }
            for (int b = 0; b < B; ++b) {
                if (!M[b]) continue;
                P[b].n_cg += ncg[b];
                P[b].n_pcg += npcg[b];
                P[b].n_green += step_greens[b];
                // a step begun by this round's commit starts from these counts
                if (P[b].recount) mark_counters(P[b]);
            }
            std::vector<int> failed(B, 0);
            for (int b = 0; b < B; ++b) failed[b] = M[b] && rc[b] != RVE_OK;
            if (any(failed)) {
                CHK(set_mask(1, failed));
                HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, B, dmask[1], st));
                for (int b = 0; b < B; ++b)
                    if (failed[b]) CHK(on_failure(b, P[b], rc[b], why_[b], fresh));
            }
        }
        int worst = RVE_OK;
        for (int b = 0; b < B; ++b) {
            const Progress& q = P[b];
            if (status) status[b] = q.status;
            if (worst == RVE_OK && q.status != RVE_OK) worst = q.status;
            if (!info) continue;
            rve_step_info o;
            std::memset(&o, 0, sizeof(o));
            if (q.has_last) {
                o = q.last;
            } else {
                const SlotState& S0 = slots[b];
                o.E = S0.E; o.Sigma = S0.Sigma; o.tau = S0.tau; o.T = S0.T;
                o.fractured = S0.fractured ? 1 : 0;
                o.step = S0.step;
                o.G_inst = NAN;
            }
            o.n_stagger = q.n_stag;
            o.n_cg = q.n_cg;
            o.n_pcg = q.n_pcg;
            o.n_greenop = q.n_green;
            o.n_steps = q.n_steps;
            o.n_substeps = q.n_sub;
            o.reason = q.reason;
            info[b] = o;
        }
        return worst;
    }

    // One stagger iteration for the slots in S after their equilibrium solve:
    // (A) the load E with D(phi(E)) = tau, (U) the convergence test on the
    // relative changes of phi and E, and the next working damage (Anderson
    // mixing of the iterates, or the plain fixed-point step).
    int stagger_iteration(const std::vector<int>& S, std::vector<Progress>& P, std::vector<int>& rc,
                          std::vector<int>& npcg) {
        std::vector<double> tau(B, 0.0), E(B, 0.0), En(B, 0.0);
        for (int b = 0; b < B; ++b)
            if (S[b]) { tau[b] = P[b].tau; E[b] = P[b].E; }
        CHK(set_mask(1, S));
        HIPCHK(launch_copy<T>(phi_w, px, g.N, B, dmask[1], st));
        if (phi64) HIPCHK(launch_widen<T>(phi_w, phi64, g.N, B, dmask[1], st));
        CHK(arclength(tau, E, px, S, En, npcg, rc));
        HIPCHK(launch_diff_norms<T>(px, phi_w, g.N, B, partials, nred, dmask[1], st));
        HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, dmask[1], st));
        CHK(read_sums(2));
        std::vector<int> take(B, 0), mixing(B, 0);
        for (int b = 0; b < B; ++b) {
            if (!S[b]) continue;
            Progress& q = P[b];
            q.it += 1;
            q.n_stag += 1;
            if (rc[b] != RVE_OK) continue;
            const double dphi = std::sqrt(sum_of(b, 0)) / std::max(std::sqrt(sum_of(b, 1)), 1e-300);
            const double dEr = std::fabs(En[b] - q.E) / std::max(std::fabs(En[b]), 1e-300);
            const double err = std::max(dphi, dEr);
            if (trace)
                std::fprintf(stderr, "[mirve] slot %d step %d stagger %d dphi %.3e dE %.3e E %.9g\n",
                             b, slots[b].step + 1, q.it, dphi, dEr, En[b]);
            q.E = En[b];
            if (err < 0.5 * q.ref) { q.ref = err; q.ref_it = q.it; }
            if (!std::isfinite(err)) {
                slot_fail(rc, b, RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "non-finite stagger update");
            } else if (err < cfg.tol ||
                       (sizeof(T) < sizeof(double) && err < kFloorFactor * cfg.tol &&
                        q.it - q.ref_it >= kFloorWindow)) {
                // converged; in mixed precision also when the error has come
                // within kFloorFactor of tol and has not halved for
                // kFloorWindow iterations: the FP32 mechanics solve gives the
                // staggered map a noise floor of that order
                take[b] = 1;
                q.stage = 2;
            } else if (q.it >= cfg.max_stagger ||
                       (cfg.stall_window > 0 && q.it - q.ref_it >= cfg.stall_window)) {
                slot_fail(rc, b, RVE_ENOCONV, RVE_WHY_STAGGER,
                          q.it >= cfg.max_stagger ? "stagger did not converge within max_stagger"
                                                  : "stagger stalled (no halving of its error within stall_window)");
            } else if (m1_max > 1) {
                mixing[b] = 1;
            } else {
                take[b] = 1;
            }
        }
        // converged, or no mixing: phi_w = phi(E)
        if (any(take)) {
            CHK(set_mask(2, take));
            HIPCHK(launch_copy<T>(px, phi_w, g.N, B, dmask[2], st));
        }
        if (!any(mixing)) return RVE_OK;
        // push F = phi(E) - phi_w and G = phi(E) into each slot's ring
        for (int ring = 0; ring < m1_max; ++ring) {
            std::vector<int> ms(B, 0);
            bool a = false;
            for (int b = 0; b < B; ++b)
                if (mixing[b] && P[b].nhist % m1_max == ring) { ms[b] = 1; a = true; }
            if (!a) continue;
            CHK(set_mask(2, ms));
            T* Fs = aF + (long long)ring * g.N * B;
            T* Gs = aG + (long long)ring * g.N * B;
            HIPCHK(launch_sub<T>(px, phi_w, Fs, g.N, B, dmask[2], st));
            HIPCHK(launch_copy<T>(px, Gs, g.N, B, dmask[2], st));
        }
        std::vector<int> mix2(B, 0), first(B, 0), nh(B, 0);
        for (int b = 0; b < B; ++b) {
            if (!mixing[b]) continue;
            P[b].nhist += 1;
            nh[b] = P[b].nhist;
            if (P[b].nhist >= 2) mix2[b] = 1;
            else first[b] = 1;
        }
        if (any(first)) {
            CHK(set_mask(2, first));
            HIPCHK(launch_copy<T>(px, phi_w, g.N, B, dmask[2], st));
        }
        if (any(mix2)) CHK(anderson_mix(mix2, nh, phi_w, rc));
        return RVE_OK;
    }

    // Commit the slots in C after the final equilibrium at their converged
    // damage (S1, s2: its unit-load stress sums): residuals of Eq. 24, history
    // (Eq. 38), committed fields, dissipation, fracture test, the trapezoid of
    // Eq. 33; then each slot's next sub-step or step.
    int commit(const std::vector<int>& C, const std::vector<double>& S1, const std::vector<double>& s2,
               std::vector<Progress>& P, std::vector<int>& fresh) {
        std::vector<double> E(B, 0.0), R1(B, 0.0), R2(B, 0.0), D(B, 0.0), G(B, 0.0);
        for (int b = 0; b < B; ++b)
            if (C[b]) E[b] = P[b].E;
        CHK(set_mask(1, C));
        // residuals of the committed state: R1 (equilibrium) and R2 (damage with
        // the H of the last damage solve)
        CHK(green(phi_w, x, 1.0, nullptr, 1.0, cgpB, dmask[1]));
        HIPCHK(launch_sum_rows(cgpB, nbx, B, sums, 0, st));
        CHK(read_sums(1));
        for (int b = 0; b < B; ++b)
            if (C[b]) R1[b] = std::sqrt(sum_of(b, 0)) / std::max(std::sqrt(s2[b]), 1e-300);
        HIPCHK(launch_damage_residual<T>(g, mat_id, mat, H, phi_w, partials, nred, dmask[1], st));
        HIPCHK(launch_sum_partials(partials, nred, 2, B, sums, dmask[1], st));
        CHK(read_sums(2));
        for (int b = 0; b < B; ++b)
            if (C[b]) R2[b] = std::sqrt(sum_of(b, 0)) / std::max(std::sqrt(sum_of(b, 1)), 1e-300);
        CHK(upload_doubles(dE, E));
        HIPCHK(launch_commit_history<T>(g, psi1, psi_ini, dE, cfg.history, Hn, dmask[1], st));
        HIPCHK(launch_copy<T>(phi_w, phi_c, g.N, B, dmask[1], st));
        HIPCHK(launch_copy<T>(x, x_c, g.s * g.N, B, dmask[1], st));
        CHK(dissip(phi_c, 1));
        for (int b = 0; b < B; ++b)
            if (C[b]) { D[b] = sum_of(b, 0) * hd_(); G[b] = sum_of(b, 1) * hd_(); }
        HIPCHK(launch_zero_int(count, B, st));
        HIPCHK(launch_fracture_count<T>(g, mat_id, mat, phi_c, cfg.frac_threshold, load_axis, count,
                                        dmask[1], st));
        HIPCHK(hipMemcpyAsync(h_count, count, sizeof(int) * B, hipMemcpyDeviceToHost, st));
        CHK(drain());
        for (int b = 0; b < B; ++b) {
            if (!C[b]) continue;
            Progress& q = P[b];
            SlotState& Ss = slots[b];
            step_greens[b] += 1;       // the R1 check
            const double Sigma = E[b] * S1[b];
            // dissipated energy per volume on the curve, T - 1/2 Sigma E, before the step
            const double dext_prev = Ss.T - 0.5 * Ss.Sigma * Ss.E;
            Ss.T += 0.5 * (Sigma + Ss.Sigma) * (E[b] - Ss.E);
            Ss.sig_max_prev = std::max(Ss.sig_max_prev, Ss.Sigma);
            Ss.E = E[b];
            Ss.Sigma = Sigma;
            Ss.tau = q.tau;
            Ss.step += 1;
            Ss.fractured = h_count[b] == 0;
            rve_step_info& o = q.last;
            std::memset(&o, 0, sizeof(o));
            o.E = E[b];
            o.Sigma = Sigma;
            o.D = D[b];
            o.Gamma = G[b];
            o.tau = q.tau;
            o.T = Ss.T;
            o.res_R1 = R1[b];
            o.res_R2 = R2[b];
            o.res_R3 = std::fabs(D[b] - q.tau) / q.tau;
            o.fractured = Ss.fractured ? 1 : 0;
            o.step = Ss.step;
            // instantaneous energy release rate (Eq. 34) on the dissipated part
            // of the curve; NaN when the crack surface did not grow
            const double dGam = G[b] - Ss.Gamma;
            o.G_inst = dGam > 0.0 ? Ss.V * ((Ss.T - 0.5 * Sigma * E[b]) - dext_prev) / dGam : NAN;
            Ss.Gamma = G[b];
            q.has_last = true;
            q.n_sub += 1;
            q.sub_done = true;
            q.pend.pop_front();
            if (!q.pend.empty()) {     // the next sub-step of this step
                begin_attempt(b, q, fresh);
                continue;
            }
            q.n_steps += 1;
            q.todo -= 1;
            q.snap = false;
            q.s_phi.clear(); q.s_H.clear(); q.s_x.clear(); q.s_tan.clear();
            if (q.todo > 0 && !(q.stop_frac && Ss.fractured)) {
                begin_step(q);
                q.recount = true;      // the round's counts are added after this
                begin_attempt(b, q, fresh);
            } else {
                q.stage = 0;
            }
        }
        return RVE_OK;
    }

    // ---- monolithic Newton-Raphson step (Sec. 4.1, Eq. 22-31) -----------------------
    // One slot, FP64, no split.  The Newton point lives in the working buffers
    // (x: the fluctuation of the actual strain, phi_w: the damage, E on the
    // host); the committed state is not touched until the commit.  Scratch
    // fields of the slot: r (J1's input strain), p (Green-operator output),
    // pp (dphi), pq (damage operator output), pb (g' dH), pz (zero damage),
    // H (the history of the Newton point).  The Krylov vectors live in the
    // caller's workspace.
    static long long nr_ld(const Geom& g) {
        const long long n = (long long)(g.s + 1) * g.N + 1;
        return (n + 31) / 32 * 32;
    }
    // workspace: V (m + 1 vectors), b, dq, J dq, the projected argument of J,
    // the dot-product partials, the Gram-Schmidt coefficients (two passes), the
    // least-squares solution, the update norms, then the rotated Hessenberg
    // columns, the rotations, the rotated right-hand side and the residual
    // estimates
    size_t nr_doubles(long long ld, int m) const {
        return (size_t)(m + 5) * ld + (size_t)(m + 5) * 64 + 3 * (size_t)(m + 2) + 8 +
               (size_t)(m + 1) * m + 2 * (size_t)m + (size_t)(m + 1) + (size_t)m +
               (sizeof(MatEntry<double>) + 7) / 8 + ((size_t)B * g.N * sizeof(uint16_t) + 7) / 8;
    }
    size_t newton_workspace(int m) const override {
        if (m < 1) return 0;
        return sizeof(double) * nr_doubles(nr_ld(g), m);
    }

    int newton_step(int slot, double dtau, const rve_newton_opts& op, void* wsp, size_t wsb,
                    rve_step_info* info) override {
        if constexpr (!std::is_same<T, double>::value) {
            (void)slot; (void)dtau; (void)op; (void)wsp; (void)wsb; (void)info;
            return fail(RVE_EINVAL, "the Newton step runs on FP64 handles only");
        } else {
            CHK(check_slot(slot));
            CHK(drop_kept(slot));
            if (cfg.split != RVE_SPLIT_NONE) return fail(RVE_EINVAL, "the Newton step takes the law without split");
            if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(RVE_EINVAL, "dtau must be finite and > 0");
            const int m = op.restart;
            if (m < 1 || m > 1000 || op.max_cycles < 1 || op.max_newton < 1 || !(op.krylov_tol > 0.0) ||
                !(op.theta > 0.0 && op.theta <= 1.0))
                return fail(RVE_EINVAL, "invalid Newton options");
            if (!wsp || wsb < newton_workspace(m)) return fail(RVE_EINVAL, "Newton workspace too small");
            const double tol = op.tol > 0.0 ? op.tol : cfg.tol;
            Range rg("mirve: rve_step_newton (Eq. 22-31)");
            const int b = slot;
            const long long N = g.N, sN = (long long)g.s * N, n = sN + N + 1, ld = nr_ld(g);
            double* V = (double*)wsp;
            double* bv = V + (long long)(m + 1) * ld;
            double* dq = bv + ld;
            double* tv = dq + ld;
            double* part = tv + ld;
            double* hA = part + (long long)(m + 5) * 64;
            double* hB = hA + (m + 2);
            double* cf = hB + (m + 2);
            double* upd = cf + (m + 2);
            double* Rm = upd + 8;
            double* csd = Rm + (long long)(m + 1) * m;
            double* snd = csd + m;
            double* gvd = snd + m;
            double* est = gvd + (m + 1);
            double* pv = est + m;                  // [P v_x, v_phi, v_E] (ld doubles)
            MatEntry<T>* idm = reinterpret_cast<MatEntry<T>*>(pv + ld);
            uint16_t* zid = reinterpret_cast<uint16_t*>(pv + ld + (sizeof(MatEntry<double>) + 7) / 8);
            double* xs = x + b * sN;
            double* ph = phi_w + b * N;
            double* Hb = H + b * N;
            SlotState& S = slots[b];
            const double tau = S.tau + dtau;
            const double hd = hd_();
            step_greens.assign(B, 0);
            F6 f;
            for (int c = 0; c < 6; ++c) f.v[c] = c < g.s ? cfg.f[c] : 0.0;
            CHK(set_mask(0, only(b)));
            HIPCHK(launch_copy<T>(phi_c, phi_w, N, B, dmask[0], st));
            HIPCHK(launch_fill<T>(pz, T(0), N, B, dmask[0], st));
            {   // the identity material (reference medium of P) for every voxel
                MatEntry<T> me;
                std::memset(&me, 0, sizeof(me));
                for (int a = 0; a < g.s; ++a) me.C[a * g.s + a] = T(1);
                me.K = T(1.0 / 3.0);
                me.Gc = T(1);
                me.drive = T(1);
                CHK(upload_bytes(idm, &me, sizeof(me)));
                HIPCHK(launch_zero_int(reinterpret_cast<int*>(zid), (int)(((long long)B * N * 2 + 3) / 4), st));
            }
            rve_step_info o;
            std::memset(&o, 0, sizeof(o));
            auto give_up = [&](int code, int why, const char* msg) {
                if (info) {
                    o.E = S.E; o.Sigma = S.Sigma; o.tau = S.tau; o.T = S.T; o.step = S.step;
                    o.fractured = S.fractured ? 1 : 0;
                    o.G_inst = NAN;
                    o.n_greenop = step_greens[b];
                    o.reason = why;
                    *info = o;
                }
                return fail(code, msg);
            };
            // the starting point: E x_c, or from the unloaded state the elastic
            // unit-load solution scaled to the first guess of E
            double E = S.E;
            if (E == 0.0) {
                HIPCHK(launch_copy<T>(x_c, x, sN, B, dmask[0], st));
                std::vector<int> its(B, 0), rcs(B, RVE_OK);
                CHK(mech_solve(phi_w, 0, only(b), its, rcs));
                o.n_cg += its[b];
                if (rcs[b] != RVE_OK) return give_up(rcs[b], RVE_WHY_CG, "mechanics of the first guess failed");
                CHK(unit_response(phi_w, 0));
                HIPCHK(launch_max_field<T>(psi1, N, B, partials, nred, dmask[0], st));
                HIPCHK(launch_max_partials(partials, nred, B, sums, dmask[0], st));
                CHK(read_sums(1));
                const double pm = sum_of(b, 0);
                E = pm > 0.0 ? std::sqrt(S.min_gc / cfg.ell / pm) : 1.0;
                HIPCHK(launch_axpby(sN, E, xs, 0.0, xs, st));
            } else {
                HIPCHK(launch_axpby(sN, E, x_c + b * sN, 0.0, xs, st));
            }
            // relaxation of Eq. 31 (1 for the first two steps)
            double alpha = 1.0;
            if (op.relax && S.step >= 2 && S.sig_max_prev > 0.0)
                alpha = std::max(op.theta, std::min(1.0, S.Sigma / S.sig_max_prev));
            NrArgs a;
            std::memset(&a, 0, sizeof(a));
            a.g = g;
            a.mat_id = mat_id + b * N;
            a.mat = mat + (long long)b * g.mstride;
            a.f = f;
            a.x = xs;
            a.E = E;
            a.phi = ph;
            a.psi_ini = psi_ini + b * N;
            a.Hn = Hn + b * N;
            a.history = cfg.history;
            const double inv_g0 = 1.0 / (1.0 + g.k_res);
            auto read = [&](const double* dev, double* hostp, long long cnt) -> int {
                HIPCHK(hipMemcpyAsync(hostp, dev, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
                return drain();
            };
            // bv = -R(q) (Eq. 24); returns D(phi)
            auto residual = [&](double& D) -> int {
                a.E = E;
                HIPCHK(launch_nr_history(a, Hb, st));
                CHK(green(phi_w, x, E, p, 1.0, cgpB, dmask[0]));
                step_greens[b] += 1;
                HIPCHK(launch_pcg_matvec<T>(g, mat_id, mat, H, 0, 0.0, phi_w, pq, nullptr, nred, nullptr,
                                            dmask[0], st));
                CHK(dissip(phi_w, 0));
                D = sum_of(b, 0) * hd;
                HIPCHK(launch_nr_pack(sN, N, bv, p + b * sN, -1.0, pq + b * N, -1.0, Hb, 2.0, nullptr, 0.0,
                                      tau - D, st));
                return RVE_OK;
            };
            // outx = P vx, the projection on compatible strains: the Green
            // operator of the identity material at phi = 0, divided by g(0)
            auto project = [&](const double* vx, double* outx) -> int {
                HIPCHK(launch_axpby(sN, 1.0, vx, 0.0, r + b * sN, st));
                ov_mid = zid;
                ov_mat = idm;
                const int rc = green(pz, r, 0.0, p, inv_g0, cgpB, dmask[0]);
                ov_mid = nullptr;
                ov_mat = nullptr;
                CHK(rc);
                step_greens[b] += 1;
                HIPCHK(launch_axpby(sN, 1.0, p + b * sN, 0.0, outx, st));
                return RVE_OK;
            };
            // out = J(q) v (Eq. 25)
            auto jac = [&](const double* v, double* out) -> int {
                HIPCHK(launch_nr_jac_point(a, v, inv_g0, r + b * sN, pp + b * N, pb + b * N, st));
                CHK(green(pz, r, 0.0, p, 1.0, cgpB, dmask[0]));
                step_greens[b] += 1;
                HIPCHK(launch_pcg_matvec<T>(g, mat_id, mat, H, 0, 0.0, pp, pq, nullptr, nred, nullptr,
                                            dmask[0], st));
                HIPCHK(launch_dissipation_dir<T>(g, mat_id, mat, phi_w, pp, partials, nred, dmask[0], st));
                HIPCHK(launch_sum_partials(partials, nred, 1, B, sums, dmask[0], st));
                HIPCHK(launch_nr_pack(sN, N, out, p + b * sN, 1.0, pq + b * N, 1.0, pb + b * N, 1.0,
                                      sums + (long long)b * kMaxVals, hd, 0.0, st));
                return RVE_OK;
            };
            // the operator of the Newton systems: J on the compatible part of
            // the strain, the identity on the rest (J alone is singular on the
            // full strain space: J1 sees only the compatible part)
            auto jac_full = [&](const double* v, double* out) -> int {
                CHK(project(v, pv));
                HIPCHK(launch_axpby(N + 1, 1.0, v + sN, 0.0, pv + sN, st));
                CHK(jac(pv, out));
                HIPCHK(launch_axpby(sN, 1.0, v, 1.0, out, st));
                HIPCHK(launch_axpby(sN, -1.0, pv, 1.0, out, st));
                return RVE_OK;
            };
            // restarted GMRES for J dq = bv from dq = 0: classical Gram-Schmidt
            // with one reorthogonalization, the Givens rotations on the device;
            // the host reads the residual estimates every kChunk iterations.
            // Converged at a true residual <= krylov_tol |bv|; near Newton's
            // solution |bv| is so small that the rounding of the Jacobian
            // products sets a floor above that, so a restart cycle that no
            // longer halves the true residual ends the solve too, if the
            // residual is below sqrt(krylov_tol) |bv| (the Newton test of
            // Eq. 30 still decides convergence).
            constexpr int kChunk = 8;
            std::vector<double> estv(kChunk);
            auto gmres = [&](int& iters, bool& ok) -> int {
                ok = false;
                HIPCHK(launch_axpby(n, 0.0, bv, 0.0, dq, st));
                double bn2 = 0.0;
                HIPCHK(launch_mdot(bv, ld, 1, bv, n, part, hA, st));
                CHK(read(hA, &bn2, 1));
                const double bn = std::sqrt(bn2);
                if (!std::isfinite(bn)) return RVE_OK;
                if (bn == 0.0) { ok = true; return RVE_OK; }
                double prev = INFINITY;
                for (int cyc = 0; cyc <= op.max_cycles; ++cyc) {
                    // V_0 = bv - J dq (the true residual of the current dq)
                    if (cyc == 0) {
                        HIPCHK(launch_axpby(n, 1.0, bv, 0.0, V, st));
                    } else {
                        CHK(jac_full(dq, tv));
                        HIPCHK(launch_axpby(n, 1.0, bv, 0.0, V, st));
                        HIPCHK(launch_axpby(n, -1.0, tv, 1.0, V, st));
                    }
                    double beta2 = 0.0;
                    HIPCHK(launch_mdot(V, ld, 1, V, n, part, hA, st));
                    CHK(read(hA, &beta2, 1));
                    const double beta = std::sqrt(beta2);
                    if (trace) std::fprintf(stderr, "gmres cycle %d residual %.3e\n", cyc, beta / bn);
                    if (!std::isfinite(beta)) return RVE_OK;
                    if (beta <= op.krylov_tol * bn) { ok = true; return RVE_OK; }
                    if (beta > 0.5 * prev && beta <= std::sqrt(op.krylov_tol) * bn) { ok = true; return RVE_OK; }
                    prev = beta;
                    if (cyc == op.max_cycles) return RVE_OK;
                    HIPCHK(launch_gmres_start(gvd, m, hA, st));
                    HIPCHK(launch_unit_scale(V, n, hA, st));
                    int k = 0;
                    bool done = false;
                    for (int j0 = 0; j0 < m && !done; j0 += kChunk) {
                        const int j1 = std::min(m, j0 + kChunk);
                        for (int j = j0; j < j1; ++j) {
                            double* vj1 = V + (long long)(j + 1) * ld;
                            CHK(jac_full(V + (long long)j * ld, vj1));
                            HIPCHK(launch_mdot(V, ld, j + 1, vj1, n, part, hA, st));
                            HIPCHK(launch_maxpy(V, ld, j + 1, hA, -1.0, vj1, n, st));
                            HIPCHK(launch_mdot(V, ld, j + 1, vj1, n, part, hB, st));
                            HIPCHK(launch_maxpy(V, ld, j + 1, hB, -1.0, vj1, n, st));
                            HIPCHK(launch_mdot(vj1, ld, 1, vj1, n, part, hB + j + 1, st));
                            HIPCHK(launch_unit_scale(vj1, n, hB + j + 1, st));
                            HIPCHK(launch_gmres_col(j, m + 1, hA, hB, Rm, csd, snd, gvd, est, st));
                            iters += 1;
                        }
                        CHK(read(est + j0, estv.data(), j1 - j0));
                        k = j1;
                        for (int j = j0; j < j1; ++j) {
                            if (!std::isfinite(estv[j - j0])) { k = j; done = true; break; }
                            if (estv[j - j0] <= op.krylov_tol * bn) { k = j + 1; done = true; break; }
                        }
                    }
                    if (k == 0) return RVE_OK;          // breakdown at the first column
                    HIPCHK(launch_gmres_solve(k, m + 1, Rm, gvd, cf, st));
                    HIPCHK(launch_maxpy(V, ld, k, cf, 1.0, dq, n, st));
                }
                return RVE_OK;
            };
            int it = 0, nkry = 0;
            bool conv = false;
            double D = 0.0;
            for (it = 1; it <= op.max_newton; ++it) {
                CHK(residual(D));
                bool ok = false;
                CHK(gmres(nkry, ok));
                if (!ok) {
                    o.n_stagger = it; o.n_cg += nkry;
                    return give_up(RVE_ENOCONV, RVE_WHY_GMRES, "GMRES of a Newton system did not converge");
                }
                CHK(project(dq, dq));      // the strain update is compatible
                double dEh = 0.0;
                CHK(read(dq + sN + N, &dEh, 1));
                const double En = E + alpha * dEh;
                double u4[4];
                HIPCHK(launch_nr_update(g.s, N, dq, alpha, f, En, xs, ph, part, upd, st));
                CHK(read(upd, u4, 4));
                E = En;
                CHK(dissip(phi_w, 0));
                D = sum_of(b, 0) * hd;
                const double err = std::max({std::sqrt(u4[0]) / std::max(std::sqrt(u4[1]), 1e-300),
                                             std::sqrt(u4[2]) / std::max(std::sqrt(u4[3]), 1e-300),
                                             std::fabs(D - tau) / tau});
                if (!std::isfinite(err) || !std::isfinite(E)) {
                    o.n_stagger = it; o.n_cg += nkry;
                    return give_up(RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "non-finite Newton iterate");
                }
                if (trace) std::fprintf(stderr, "newton it %d E %.17g D-tau %.3e err %.3e krylov %d\n", it, E,
                                        D - tau, err, nkry);
                if (err < tol) { conv = true; break; }
            }
            if (!conv) {
                o.n_stagger = op.max_newton; o.n_cg += nkry;
                return give_up(RVE_ENOCONV, RVE_WHY_NEWTON, "Newton did not converge");
            }
            if (!(E > 0.0)) return give_up(RVE_ENUMERIC, RVE_WHY_BREAKDOWN, "Newton reached E <= 0");
            // commit (Eq. 33, 38): the history of the Newton point, then the unit
            // fluctuation x / E and the unit response the commit prices Sigma with
            a.E = E;
            HIPCHK(launch_nr_history(a, Hb, st));
            HIPCHK(launch_axpby(sN, 1.0 / E, xs, 0.0, xs, st));
            CHK(unit_response(phi_w, 0));
            std::vector<double> S1(B, 0.0), s2(B, 0.0);
            S1[b] = sum_of(b, 0) / double(N);
            s2[b] = sum_of(b, 1);
            std::vector<Progress> P(B);
            Progress& q = P[b];
            q.E = E;
            q.tau = tau;
            q.dtau = dtau;
            q.todo = 1;
            begin_step(q);
            q.stage = 2;
            std::vector<int> C = only(b), fresh(B, 0);
            CHK(commit(C, S1, s2, P, fresh));
            slope_warm[b] = 0;
            if (info) {
                o = q.last;
                o.n_stagger = it;
                o.n_cg += nkry;
                o.n_greenop = step_greens[b];
                o.n_steps = 1;
                o.n_substeps = 1;
                o.reason = RVE_WHY_NONE;
                *info = o;
            }
            return RVE_OK;
        }
    }

    // ---- single-slot helpers --------------------------------------------------------
    int check_slot(int slot) {
        if (slot < 0 || slot >= B) return fail(RVE_EINVAL, "slot out of range");
        if (!slots[slot].ready) return fail(RVE_ESTATE, "set_microstructure first");
        return RVE_OK;
    }
    std::vector<int> only(int slot) {
        std::vector<int> v(B, 0);
        v[slot] = 1;
        return v;
    }

    int get_field(int slot, int which, double* hostp, size_t cnt) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        const size_t N = (size_t)g.N, sN = (size_t)g.s * g.N;
        const long long so = (long long)slot * g.N;
        switch (which) {
            case RVE_FIELD_PHI: if (cnt != N) break; return download(hostp, phi_c + so, N);
            case RVE_FIELD_HIST: if (cnt != N) break; return download(hostp, Hn + so, N);
            case RVE_FIELD_PSI_INI: if (cnt != N) break; return download(hostp, psi_ini + so, N);
            case RVE_FIELD_PSI1: if (cnt != N) break; return download(hostp, psi1 + so, N);
            case RVE_FIELD_PHI_INI: if (cnt != N) break; return download(hostp, phi_ini + so, N);
            case RVE_FIELD_EPS1:
            case RVE_FIELD_SIG1: {
                if (cnt != sN) break;
                CHK(set_mask(0, only(slot)));
                // x holds the working strain; show the committed one
                HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, B, dmask[0], st));
                CHK(unit_response(phi_c, 0, r, p));
                return download(hostp, (which == RVE_FIELD_EPS1 ? r : p) + so * g.s, sN);
            }
            default: return fail(RVE_EINVAL, "unknown field");
        }
        return fail(RVE_EINVAL, "field size mismatch");
    }

    int set_field(int slot, int which, const double* hostp, size_t cnt) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        const size_t N = (size_t)g.N;
        const long long so = (long long)slot * g.N;
        if (cnt != N) return fail(RVE_EINVAL, "field size mismatch");
        for (size_t i = 0; i < N; ++i)
            if (!std::isfinite(hostp[i])) return fail(RVE_EINVAL, "non-finite field value");
        CHK(drain());
        switch (which) {
            case RVE_FIELD_PHI: {          // the committed crack surface follows phi
                CHK(upload(phi_c + so, hostp, N));
                CHK(set_mask(0, only(slot)));
                CHK(dissip(phi_c, 0));
                slots[slot].Gamma = sum_of(slot, 1) * hd_();
                return RVE_OK;
            }
            case RVE_FIELD_HIST: return upload(Hn + so, hostp, N);
            case RVE_FIELD_PSI1: return upload(psi1 + so, hostp, N);
            default: return fail(RVE_EINVAL, "field is read-only");
        }
    }

    int apply_green(int slot, const double* eps, double* outp) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        const size_t sN = (size_t)g.s * g.N;
        const long long fo = (long long)slot * g.s * g.N;
        CHK(drain());
        CHK(upload(r + fo, eps, sN));
        CHK(set_mask(0, only(slot)));
        CHK(green(phi_c, r, 0.0, p, 1.0, cgpB, dmask[0]));
        return download(outp, p + fo, sN);
    }

    // mask `which` = the slots that hold a microstructure, written straight
    // into the pinned staging ring (no host container)
    int set_mask_ready(int which) {
        const size_t n = sizeof(int) * B, need = (n + 255) & ~size_t(255);
        if (stage_off + need > stage_bytes) CHK(drain());
        int* slot = reinterpret_cast<int*>((char*)h_stage + stage_off);
        for (int b = 0; b < B; ++b) slot[b] = slots[b].ready ? 1 : 0;
        HIPCHK(hipMemcpyAsync(dmask[which], slot, n, hipMemcpyHostToDevice, st));
        stage_off += need;
        return RVE_OK;
    }

    int apply_green_device(const void* eps, void* outp, int repeat) override {
        CHK(set_mask_ready(0));
        for (int i = 0; i < repeat; ++i)
            CHK(green(phi_c, (const T*)eps, 0.0, (T*)outp, 1.0, cgpB, dmask[0]));
        return RVE_OK;
    }

    // The same with the spectrum and the pass partials in the caller's
    // scratch `scr` of `cap` bytes instead of the workspace (the handle's own
    // buffers are put back afterwards).
    int apply_green_device_scratch(void* scr, size_t cap, const void* eps, void* outp,
                                   int repeat) override {
        const size_t spec_b = (sizeof(cplx<T>) * g.s * (size_t)g.Nspec * B + 255) & ~size_t(255);
        const size_t part_b = sizeof(double) * (size_t)pass_blocks_max() * B;
        if (spec_b + part_b > cap)
            return fail(RVE_ENOSPC, "the handle needs " + std::to_string(spec_b + part_b) +
                                        " bytes of static scratch; the array holds " +
                                        std::to_string(cap));
        cplx<T>* const own_spec = spec;
        double* const own_part = cgpB;
        spec = reinterpret_cast<cplx<T>*>(scr);
        cgpB = reinterpret_cast<double*>((char*)scr + spec_b);
        const int rc = apply_green_device(eps, outp, repeat);
        spec = own_spec;
        cgpB = own_part;
        return rc;
    }

    int solve_mechanics(int slot, int* it, double* Sigma1) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        std::vector<int> one = only(slot), its(B, 0), rcs(B, RVE_OK);
        CHK(set_mask(0, one));
        HIPCHK(launch_copy<T>(x_c, x, g.s * g.N, B, dmask[0], st));
        CHK(mech_solve(phi_c, 0, one, its, rcs));
        if (rcs[slot] != RVE_OK) return rcs[slot];
        CHK(unit_response(phi_c, 0));
        if (Sigma1) *Sigma1 = sum_of(slot, 0) / double(g.N);
        if (it) *it = its[slot];
        HIPCHK(launch_copy<T>(x, x_c, g.s * g.N, B, dmask[0], st));
        return sync();
    }

    int solve_damage(int slot, double E, double* D, int* it, int commit) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        std::vector<int> one = only(slot), its(B, 0), rcs(B, RVE_OK);
        std::vector<double> Ev(B, 0.0), Dv(B, 0.0);
        Ev[slot] = E;
        CHK(set_mask(2, one));
        HIPCHK(launch_copy<T>(phi_c, px, g.N, B, dmask[2], st));
        if (phi64) HIPCHK(launch_widen<T>(phi_c, phi64, g.N, B, dmask[2], st));
        CHK(damage_at(Ev, px, 2, one, Dv, its, rcs));
        if (rcs[slot] != RVE_OK) return rcs[slot];
        if (D) *D = Dv[slot];
        if (it) *it = its[slot];
        if (commit) HIPCHK(launch_copy<T>(px, phi_c, g.N, B, dmask[2], st));
        return sync();
    }

    int dissipation(int slot, double* D, double* G) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        CHK(set_mask(0, only(slot)));
        CHK(dissip(phi_c, 0));
        if (D) *D = sum_of(slot, 0) * hd_();
        if (G) *G = sum_of(slot, 1) * hd_();
        return RVE_OK;
    }

    // ---- checkpoints ------------------------------------------------------------
    // Blob: a header (magic, precision, grid), the slot's scalars, then the raw
    // committed fields phi, H^n, the strain fluctuation and the tangent warm
    // start, in the bulk type.
    struct StateHeader {
        uint32_t magic, word;
        int32_t dim, n[3];
        double E, Sigma, Tc, tau, tau0, Gamma, sig_max_prev;
        int32_t step, fractured, warm, pad;
    };
    static constexpr uint32_t kStateMagic = 0x3356524du;   // "MRV3"
    size_t state_bytes() const override {
        return sizeof(StateHeader) + sizeof(T) * (size_t)g.N * (3 + g.s);
    }
    int save_state(int slot, void* host, size_t bytes) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        if (!host || bytes < state_bytes()) return fail(RVE_EINVAL, "state buffer too small");
        StateHeader hdr;
        std::memset(&hdr, 0, sizeof(hdr));
        hdr.magic = kStateMagic;
        hdr.word = sizeof(T);
        hdr.dim = g.dim; hdr.n[0] = g.nx; hdr.n[1] = g.ny; hdr.n[2] = g.nz;
        const SlotState& S = slots[slot];
        hdr.E = S.E; hdr.Sigma = S.Sigma; hdr.Tc = S.T; hdr.tau = S.tau; hdr.tau0 = S.tau0;
        hdr.Gamma = S.Gamma;
        hdr.sig_max_prev = S.sig_max_prev;
        hdr.step = S.step; hdr.fractured = S.fractured ? 1 : 0; hdr.warm = slope_warm[slot];
        std::vector<char> a, b, c, d;
        CHK(save_fields(slot, a, b, c, d));
        char* o = (char*)host;
        std::memcpy(o, &hdr, sizeof(hdr)); o += sizeof(hdr);
        for (auto* v : {&a, &b, &c, &d}) { std::memcpy(o, v->data(), v->size()); o += v->size(); }
        return RVE_OK;
    }
    int load_state(int slot, const void* host, size_t bytes) override {
        CHK(check_slot(slot));
        CHK(drop_kept(slot));
        if (!host || bytes < state_bytes()) return fail(RVE_EINVAL, "state buffer too small");
        StateHeader hdr;
        std::memcpy(&hdr, host, sizeof(hdr));
        if (hdr.magic != kStateMagic || hdr.word != sizeof(T) || hdr.dim != g.dim || hdr.n[0] != g.nx ||
            hdr.n[1] != g.ny || hdr.n[2] != g.nz)
            return fail(RVE_EINVAL, "state blob of another grid or precision");
        const double sc[7] = {hdr.E, hdr.Sigma, hdr.Tc, hdr.tau, hdr.tau0, hdr.Gamma, hdr.sig_max_prev};
        for (double v : sc)
            if (!std::isfinite(v)) return fail(RVE_EINVAL, "non-finite scalar in state blob");
        const size_t fN = sizeof(T) * g.N, sN = fN * g.s;
        const char* p = (const char*)host + sizeof(hdr);
        const T* fields = reinterpret_cast<const T*>(p);
        const size_t cnt = (size_t)g.N * (3 + g.s);
        for (size_t i = 0; i < cnt; ++i) {
            T v;
            std::memcpy(&v, (const char*)fields + i * sizeof(T), sizeof(T));
            if (!std::isfinite((double)v)) return fail(RVE_EINVAL, "non-finite field value in state blob");
        }
        CHK(load_fields(slot, p, p + fN, p + 2 * fN, p + 2 * fN + sN));
        SlotState& S = slots[slot];
        S.E = hdr.E; S.Sigma = hdr.Sigma; S.T = hdr.Tc; S.tau = hdr.tau; S.tau0 = hdr.tau0;
        S.Gamma = hdr.Gamma;
        S.sig_max_prev = hdr.sig_max_prev;
        S.step = hdr.step; S.fractured = hdr.fractured != 0;
        slope_warm[slot] = hdr.warm ? 1 : 0;
        return RVE_OK;
    }

    // ---- launch shape -----------------------------------------------------------
    // One-component passes (the damage preconditioner): the x passes keep the
    // rows per block of the s-component ones (the grid stays as large); the
    // axis passes take s times the lines (columns) per block, rounded down to
    // a power of two (at least 4 lines for the fixed-size FFTs, so that a
    // wave's lanes all carry butterflies).  LDS and threads are sized for one
    // component, which raises the blocks per CU.
    void one_comp_shape() {
        const size_t ce = sizeof(cplx<T>);
        // The one-component x passes take more rows per block than the
        // s-component ones where the batch still gives about 1024 blocks or
        // more: the same LDS holds s times fewer lines, the blocks carry more
        // waves, and the transposed spectrum is read and written in longer
        // runs (16 rows: 128 B in FP32).  The partial-sum buffers are sized
        // for two rows per block, so any larger count fits them.
        RB1 = RB;
        if (plx.fastN) {
            const long long rows = (long long)g.ny * g.nz;
            auto fits = [&](int rb) {
                return rb <= 16 && rb <= rows && (rb / 2) * split_max(g.nx) <= 256 &&
                       (size_t)(rb / 2) * lds_line(g.nx) * ce <= kLdsCap &&
                       rows * B / rb >= 1024;
            };
            while (fits(2 * RB1)) RB1 *= 2;
        }
        nbx1 = (int)((g.ny * (long long)g.nz + RB1 - 1) / RB1);
        if (plx.fastN) {
            thr_x1 = threads_for((RB1 / 2) * split_max(g.nx));
            lds_x1 = (size_t)(RB1 / 2) * lds_line(g.nx) * ce;
        } else {
            thr_x1 = thr_x;
            lds_x1 = lds_x;
        }
        auto lines1 = [&](const AxisPlan& pl, int tl_s, int cap, size_t lds_s, int thr_s, int& tl1,
                          size_t& lds1, int& thr1) {
            tl1 = pow2_floor(std::max(1, g.s * tl_s));
            if (!pl.fastN) {               // within the s-component shape
                lds1 = lds_s;
                thr1 = thr_s;
                return;
            }
            tl1 = std::max(tl1, 4);
            auto fits = [&](int t) {
                return t <= cap && t * split_max(pl.N) <= 256 &&
                       (size_t)t * lds_line(pl.N) * ce + axis_tw_bytes(pl.N) <= kLdsCap;
            };
            while (tl1 > 1 && !fits(tl1)) tl1 /= 2;
            lds1 = (size_t)tl1 * lds_line(pl.N) * ce + axis_tw_bytes(pl.N);
            thr1 = threads_for(tl1 * split_max(pl.N));
        };
        lines1(ply, tly, 1 << 20, lds_y, thr_y, tly1, lds_y1, thr_y1);
        if (g.dim == 3) lines1(plz, tlz, g.ny, lds_z, thr_z, tlz1, lds_z1, thr_z1);
    }

    int set_shape(const Shape& sh) {
        Geom g2;
        AxisPlan a = plx, b = ply, d = plz;
        int rb = RB, nb = nbx, mx = maxb_x, ty = tly, my = maxb_y, tz = tlz, mz = maxb_z;
        int t1 = thr_x, t2 = thr_y, t3 = thr_z;
        size_t lx = lds_x, ly = lds_y, lz = lds_z;
        std::string why;
        if (!make_geom(cfg, g2, a, b, d, rb, nb, mx, lx, ty, my, ly, tz, mz, lz, t1, t2, t3, why, &sh))
            return fail(RVE_EINVAL, why);
        a.tw_off = plx.tw_off;
        b.tw_off = ply.tw_off;
        d.tw_off = plz.tw_off;
        plx = a; ply = b; plz = d;
        RB = rb; nbx = nb; maxb_x = mx; lds_x = lx;
        tly = ty; maxb_y = my; lds_y = ly;
        tlz = tz; maxb_z = mz; lds_z = lz;
        thr_x = t1; thr_y = t2; thr_z = t3;
        if (sh.nt >= 0 && cfg.streaming < 0) stream_nt = sh.nt ? 1 : 0;   // a fixed policy wins
        if (sh.yblock >= 0) y_block = sh.yblock;
        one_comp_shape();
        clear_graphs();            // captured launches carry the old shape
        return RVE_OK;
    }

    // Autotuner: time the CG-mode passes of every feasible launch shape on the
    // slots' own data and keep the fastest: rows per block of the x passes
    // (one value for x-forward and x-inverse, which share their partials),
    // lines per block of the y pass, y columns per tile of the z pass.  The
    // choice is cached per (grid, batch, precision) for the process.
    int autotune(int repeat, int* out) override {
        CHK(drop_kept(-1));
        bool ready = false;
        for (int b = 0; b < B; ++b) ready = ready || slots[b].ready;
        if (!ready) return fail(RVE_ESTATE, "set_microstructure first");
        repeat = std::max(1, repeat);
        char key[128];
        std::snprintf(key, sizeof(key), "%d:%dx%dx%d:B%d:w%d:s%d", g.dim, g.nx, g.ny, g.nz, B,
                      (int)sizeof(T), cfg.streaming);
        {
            std::lock_guard<std::mutex> lk(tune_mutex());
            auto it = tune_cache().find(key);
            if (it != tune_cache().end()) {
                CHK(set_shape(it->second));
                if (out) { out[0] = RB; out[1] = y_lines_out(); out[2] = tlz; out[3] = stream_nt; }
                return RVE_OK;
            }
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto timed = [&](int pass, double& us) -> int {
            CHK(profile_pass(pass, 2, nullptr));
            HIPCHK(hipEventRecord(e0, st));
            CHK(profile_pass(pass, repeat, nullptr));
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            us = 1e3 * ms / repeat;
            return RVE_OK;
        };
        Shape best;
        best.rb = RB;
        best.tly = tly;
        best.tlz = g.dim == 3 ? tlz : 0;
        best.nt = stream_nt;
        best.yblock = y_block;
        double tb = INFINITY;
        for (int rb : {2, 4, 8, 16, 32}) {
            Shape sh = best;
            sh.rb = rb;
            if (set_shape(sh) != RVE_OK) continue;
            double a = 0, c = 0;
            CHK(timed(3, a));
            CHK(timed(4, c));
            if (a + c < tb) { tb = a + c; best.rb = rb; }
        }
        CHK(set_shape(best));
        tb = INFINITY;
        for (int t : {1, 2, 4, 8, 16}) {
            Shape sh = best;
            sh.tly = t;
            sh.yblock = 1;
            if (set_shape(sh) != RVE_OK) continue;
            double a = 0;
            CHK(timed(g.dim == 3 ? 5 : 1, a));
            if (a < tb) { tb = a; best.tly = t; best.yblock = 1; }
        }
        if (wave_y()) {   // the one-wave y pass against the best block shape
            Shape sh = best;
            sh.yblock = 0;
            double a = 0;
            if (set_shape(sh) == RVE_OK) {
                CHK(timed(g.dim == 3 ? 5 : 1, a));
                if (a < tb) { tb = a; best.yblock = 0; }
            }
        }
        if (g.dim == 3) {
            CHK(set_shape(best));
            tb = INFINITY;
            for (int t : {1, 2, 4, 8, 16}) {
                Shape sh = best;
                sh.tlz = t;
                if (set_shape(sh) != RVE_OK) continue;
                double a = 0;
                CHK(timed(1, a));
                if (a < tb) { tb = a; best.tlz = t; }
            }
        }
        // streaming policy of the Krylov x passes at the chosen shape
        tb = INFINITY;
        for (int nt : {0, 1}) {
            if (cfg.streaming >= 0 && nt != cfg.streaming) continue;   // fixed by the config
            Shape sh = best;
            sh.nt = nt;
            if (set_shape(sh) != RVE_OK) continue;
            double a = 0, c = 0;
            CHK(timed(3, a));
            CHK(timed(4, c));
            if (a + c < tb) { tb = a + c; best.nt = nt; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        CHK(set_shape(best));
        {
            std::lock_guard<std::mutex> lk(tune_mutex());
            tune_cache()[key] = best;
        }
        if (out) { out[0] = RB; out[1] = y_lines_out(); out[2] = tlz; out[3] = stream_nt; }
        return RVE_OK;
    }
    // The one-wave y pass applies to 128-, 256- and 512-point y lines.
    bool wave_y() const { return (g.ny == 128 || g.ny == 256 || g.ny == 512) && ply.N == g.ny; }
    // lines per block of the y pass as reported: 0 for the one-wave pass
    int y_lines_out() const { return wave_y() && !y_block ? 0 : tly; }
    static std::map<std::string, Shape>& tune_cache() {
        static std::map<std::string, Shape> m;
        return m;
    }
    static std::mutex& tune_mutex() {
        static std::mutex m;
        return m;
    }

    // Launch one kind of pass `repeat` times on every ready RVE of the batch
    // (for timing against its algorithmic bytes).  0: x-forward (constitutive),
    // 1: the projection axis pass, 2: x-inverse (store), 3: x-forward with the
    // CG updates of x and p, 4: x-inverse with the CG update of r (alpha = 0,
    // so the iterate is unchanged).
    int profile_pass(int pass, int repeat, double* bytes) override {
        CHK(drop_kept(-1));
        std::vector<int> rd(B, 0);
        int nready = 0;
        for (int b = 0; b < B; ++b) { rd[b] = slots[b].ready ? 1 : 0; nready += rd[b]; }
        if (!nready) return fail(RVE_ESTATE, "set_microstructure first");
        CHK(set_mask(0, rd));
        std::vector<CgDev> c(B);
        for (int b = 0; b < B; ++b) {
            std::memset(&c[b], 0, sizeof(CgDev));
            c[b].rr_hist[0] = c[b].rr_hist[1] = c[b].rr = c[b].bn2 = 1.0;
            c[b].max_it = -1;           // timing: alpha = 0, beta = 1/2, no stopping test
            c[b].conv = rd[b] ? kNotDone : -1;
        }
        CHK(drain());
        HIPCHK(hipMemcpy(cg, c.data(), sizeof(CgDev) * B, hipMemcpyHostToDevice));
        AxisArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.spec = spec;
        a.active = dmask[0];
        const bool three = g.dim == 3;
        a.pl = three ? plz : ply;
        a.tw = tw + (three ? plz.tw_off : ply.tw_off);
        a.contiguous = three ? 0 : 1;
        a.lines = three ? tlz : tly;
        a.threads = three ? thr_z : thr_y;
        a.block_only = y_block;
        const dim3 grid = three ? dim3((unsigned)(g.nxh * ((g.ny + tlz - 1) / tlz)), 1, B)
                                : dim3((unsigned)((g.nxh * (long long)g.nz + tly - 1) / tly), 1, B);
        for (int i = 0; i < repeat; ++i) {
            switch (pass) {
                case 0: CHK(fwd_x(XF_GREEN, phi_c, r, 0.0, cgpA, dmask[0])); break;
                case 1: HIPCHK(launch_axis<T>(a, AX_FWD_P_INV, three ? maxb_z : maxb_y, grid,
                                              three ? lds_z : lds_y, st)); break;
                case 2: CHK(inv_x(XI_STORE, p, 1.0, cgpB, dmask[0])); break;
                case 3: CHK(fwd_x(XF_CG, phi_c, nullptr, 0.0, nullptr, nullptr, 1)); break;
                case 4: CHK(inv_x(XI_CG, nullptr, 1.0, cgpB, nullptr, 1)); break;
                case 5: {   // the forward y pass of a 3D operator (2D: as pass 1)
                    AxisArgs<T> y = a;
                    y.pl = ply;
                    y.tw = tw + ply.tw_off;
                    y.contiguous = 1;
                    y.lines = tly;
                    y.threads = thr_y;
                    HIPCHK(launch_axis<T>(y, three ? AX_FWD : AX_FWD_P_INV, maxb_y, grid_y(tly), lds_y, st));
                    break;
                }
                default: return fail(RVE_EINVAL, "unknown pass");
            }
        }
        // compulsory bytes of one launch: every input read once, every output
        // written once; a half spectrum holds n_x/2 + 1 complex values per row
        const double w = sizeof(T), sp = 2.0 * g.nxh / g.nx, S = g.s, N = (double)g.N * nready;
        double bb = 0.0;
        switch (pass) {
            case 0: bb = N * ((S + 1) * w + 2) + N * sp * S * w; break;
            case 1: bb = 2.0 * N * sp * S * w; break;
            case 2: bb = N * sp * S * w + N * S * w; break;
            case 3: bb = N * (5 * S * w + w + 2) + N * sp * S * w; break;
            case 4: bb = N * sp * S * w + N * 2 * S * w; break;
            case 5: bb = 2.0 * N * sp * S * w; break;
        }
        if (bytes) *bytes = bb;
        return RVE_OK;
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
    if (!(c->h > 0) || !(c->ell > 0) || !(c->k_res > 0) || !std::isfinite(c->h) ||
        !std::isfinite(c->ell) || !std::isfinite(c->k_res)) {
        why = "h, ell, k_res must be finite and > 0";
        return RVE_EINVAL;
    }
    if (c->split != RVE_SPLIT_NONE && c->split != RVE_SPLIT_VOLDEV) { why = "bad split"; return RVE_EINVAL; }
    if (c->precision != RVE_PREC_FP64 && c->precision != RVE_PREC_MIXED) { why = "bad precision"; return RVE_EINVAL; }
    if (!(c->tol >= 0) || !(c->tol_cg >= 0) || !(c->tol_pcg >= 0) || !(c->tol_al >= 0)) {
        why = "tolerances must be >= 0 (0: the precision's default)";
        return RVE_EINVAL;
    }
    if (c->max_stagger < 1 || c->max_cg < 1 || c->max_pcg < 1) { why = "iteration limits must be >= 1"; return RVE_EINVAL; }
    if (c->max_halvings < 0 || c->max_halvings > 12) { why = "max_halvings in [0, 12]"; return RVE_EINVAL; }
    if (c->stall_window < 0) { why = "stall_window must be >= 0"; return RVE_EINVAL; }
    if (c->anderson_depth < 0 || c->anderson_depth > kAndersonMax) { why = "anderson_depth in [0, 5]"; return RVE_EINVAL; }
    if (c->max_materials < 1 || c->max_materials > kMaxMat) { why = "max_materials in [1, 65536]"; return RVE_EINVAL; }
    if (c->batch < 1 || c->batch > 1024) { why = "batch in [1, 1024]"; return RVE_EINVAL; }
    if (c->graphs != 0 && c->graphs != 1) { why = "graphs must be 0 or 1"; return RVE_EINVAL; }
    if (c->streaming < -1 || c->streaming > 1) { why = "streaming must be -1, 0 or 1"; return RVE_EINVAL; }
    if (c->damage_precond != RVE_PRECOND_FFT && c->damage_precond != RVE_PRECOND_JACOBI) {
        why = "damage_precond must be RVE_PRECOND_FFT or RVE_PRECOND_JACOBI";
        return RVE_EINVAL;
    }
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
    int RB, mx, ty, my, tz, mz, t1, t2, t3;
    size_t lx, ly, lz;
    if (!Solver<T>::make_geom(*c, g, a, b, d, RB, nbx, mx, lx, ty, my, ly, tz, mz, lz, t1, t2, t3, why))
        return RVE_EINVAL;
    return RVE_OK;
}

static thread_local std::string g_last_error;

// Static device scratch of rve_apply_green_op_device_noalloc.  Host code never
// uses its name as an address: each device's copy is found once, at the
// set-up of the first handle on that device, with that device current.
static __device__ __align__(256) unsigned char scratch[RVE_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[256];
static bool g_scratch_tried[256];

// Address of the current device's scratch array (nullptr if the runtime
// could not give it; the error text goes to why).
static void* scratch_address(std::string& why) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
        why = "no current HIP device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_tried[dev]) {
        g_scratch_tried[dev] = true;
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    if (!g_scratch_ptr[dev]) why = "the static scratch array has no address on this device";
    return g_scratch_ptr[dev];
}

// A tolerance of 0 takes the default of the precision mode.  FP32 fields
// resolve D(E) to about 1e-7, so in mixed precision the constraint is held
// to 1e-6 and the damage solves that evaluate it to 1e-7.
static void resolve_defaults(rve_config& c) {
    const bool mixed = c.precision == RVE_PREC_MIXED;
    if (c.tol == 0.0) c.tol = mixed ? 1e-5 : 1e-8;
    if (c.tol_cg == 0.0) c.tol_cg = mixed ? 1e-6 : 1e-10;
    if (c.tol_pcg == 0.0) c.tol_pcg = mixed ? 1e-10 : 1e-12;
    if (c.tol_al == 0.0) c.tol_al = mixed ? 1e-6 : 1e-10;
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
    c->tol = 0.0;          // the precision's defaults (resolve_defaults)
    c->tol_cg = 0.0;
    c->tol_pcg = 0.0;
    c->tol_al = 0.0;
    c->max_stagger = 300;
    c->max_halvings = 8;
    c->stall_window = 0;
    c->max_cg = 20000;
    c->max_pcg = 20000;
    c->anderson_depth = 5;
    c->frac_threshold = 0.95;
    c->A_g = 0.0;
    c->max_materials = 4096;
    c->batch = 1;
    c->damage_precond = RVE_PRECOND_FFT;
    c->graphs = 1;
    c->streaming = -1;
    return RVE_OK;
}

int rve_query_workspace(const rve_config* c, size_t* bytes) {
    std::string why;
    if (!bytes) return RVE_EINVAL;
    int rc = validate(c, why);
    if (rc) { g_last_error = why; return rc; }
    Geom g;
    int nbx = 1;
    Layout L;
    if (c->precision == RVE_PREC_FP64) {
        if ((rc = geom_check<double>(c, g, nbx, why))) { g_last_error = why; return rc; }
        Solver<double>::layout(*c, g, nbx, L, nullptr);
    } else {
        if ((rc = geom_check<float>(c, g, nbx, why))) { g_last_error = why; return rc; }
        Solver<float>::layout(*c, g, nbx, L, nullptr);
    }
    *bytes = L.total;
    return RVE_OK;
}

int rve_create(const rve_config* c, void* ws, size_t wsb, void* stream, rve_handle* out) {
    if (!out) return RVE_EINVAL;
    *out = nullptr;
    size_t need = 0;
    int rc;
    if ((rc = rve_query_workspace(c, &need))) return rc;
    if (!ws) { g_last_error = "null workspace"; return RVE_EINVAL; }
    if (wsb < need) { g_last_error = "workspace too small"; return RVE_ENOSPC; }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) { g_last_error = "workspace not 256-byte aligned"; return RVE_EINVAL; }
    auto* h = new rve_handle_s();
    rve_config cr = *c;
    resolve_defaults(cr);
    h->cfg = cr;
    hipStream_t st = (hipStream_t)stream;
    if (c->precision == RVE_PREC_FP64) {
        auto* s = new Solver<double>(h, cr, ws, st);
        h->impl.reset(s);
        rc = s->init_device();
    } else {
        auto* s = new Solver<float>(h, cr, ws, st);
        h->impl.reset(s);
        rc = s->init_device();
    }
    if (rc) {
        g_last_error = h->err;
        delete h;
        return rc;
    }
    // the allocation-free entry point reports a missing address itself
    std::string why;
    h->scratch = scratch_address(why);
    *out = h;
    return RVE_OK;
}

int rve_destroy(rve_handle h) {
    delete h;
    return RVE_OK;
}

int rve_batch_size(rve_handle h) { return h ? h->impl->B : 0; }

int rve_set_microstructure_slot(rve_handle h, int slot, const uint16_t* phase_id,
                                const rve_phase* phases, int nphases, const double* theta,
                                const uint8_t* void_mask, const uint8_t* phi_disc, double phi_M) {
    if (!h) return RVE_EINVAL;
    return h->impl->set_microstructure(slot, phase_id, phases, nphases, theta, nullptr, void_mask,
                                       phi_disc, phi_M);
}

int rve_set_microstructure_euler(rve_handle h, int slot, const uint16_t* phase_id,
                                 const rve_phase* phases, int nphases, const double* euler,
                                 const uint8_t* void_mask, const uint8_t* phi_disc, double phi_M) {
    if (!h || !euler) return RVE_EINVAL;
    return h->impl->set_microstructure(slot, phase_id, phases, nphases, nullptr, euler, void_mask,
                                       phi_disc, phi_M);
}

int rve_set_microstructure(rve_handle h, const uint16_t* phase_id, const rve_phase* phases,
                           int nphases, const double* theta, const uint8_t* void_mask,
                           const uint8_t* phi_disc, double phi_M) {
    return rve_set_microstructure_slot(h, 0, phase_id, phases, nphases, theta, void_mask, phi_disc,
                                       phi_M);
}

int rve_run_slots(rve_handle h, const double* dtau, const int* max_steps, int flags,
                  rve_step_info* info, int* status) {
    if (!h || !dtau || !max_steps) return RVE_EINVAL;
    if (flags & ~RVE_RUN_STOP_AT_FRACTURE) { h->err = "unknown flags"; return RVE_EINVAL; }
    return h->impl->run(dtau, max_steps, flags, info, status);
}

int rve_run_stats(rve_handle h, double* out2) {
    if (!h || !out2) return RVE_EINVAL;
    const SolverBase& s = *h->impl;
    out2[0] = double(s.run_rounds);
    out2[1] = s.run_rounds > 0 ? double(s.run_active) / (double(s.run_rounds) * s.B) : 0.0;
    return RVE_OK;
}

int rve_run_budget(rve_handle h, const double* dtau, const int* max_steps, long long total_steps, int flags,
                   rve_step_info* info, int* status) {
    if (!h || !dtau) return RVE_EINVAL;
    if (flags & ~(RVE_RUN_STOP_AT_FRACTURE | RVE_RUN_KEEP)) { h->err = "unknown flags"; return RVE_EINVAL; }
    if (total_steps < 0) { h->err = "total_steps must be >= 0"; return RVE_EINVAL; }
    const int B = h->impl->B;
    std::vector<int> todo(B, 1 << 30);
    if (max_steps)
        for (int b = 0; b < B; ++b) todo[b] = max_steps[b];
    return h->impl->run(dtau, todo.data(), flags, info, status, total_steps);
}

int rve_step_dissipation_slots(rve_handle h, const double* dtau, rve_step_info* info, int* status) {
    if (!h || !dtau) return RVE_EINVAL;
    std::vector<int> one(h->impl->B, 1);
    return h->impl->run(dtau, one.data(), 0, info, status);
}

int rve_step_dissipation(rve_handle h, double dtau, rve_step_info* out) {
    if (!h) return RVE_EINVAL;
    if (h->impl->B != 1) { h->err = "batched handle: use rve_step_dissipation_slots"; return RVE_EINVAL; }
    if (!(dtau > 0.0) || !std::isfinite(dtau)) { h->err = "dtau must be finite and > 0"; return RVE_EINVAL; }
    int status = RVE_OK, one = 1;
    int rc = h->impl->run(&dtau, &one, 0, out, &status);
    return rc != RVE_OK ? rc : status;
}

void rve_newton_default_opts(rve_newton_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 0.0;
    o->krylov_tol = 1e-12;
    o->theta = 0.3;
    o->restart = 200;
    o->max_cycles = 100;
    o->max_newton = 50;
    o->relax = 1;
}

int rve_newton_workspace(rve_handle h, int restart, size_t* bytes) {
    if (!h || !bytes) return RVE_EINVAL;
    if (restart < 1 || restart > 1000) { h->err = "restart must be in 1..1000"; return RVE_EINVAL; }
    *bytes = h->impl->newton_workspace(restart);
    return RVE_OK;
}

int rve_step_newton(rve_handle h, int slot, double dtau, const rve_newton_opts* opts, void* workspace,
                    size_t workspace_bytes, rve_step_info* info) {
    if (!h) return RVE_EINVAL;
    rve_newton_opts o;
    rve_newton_default_opts(&o);
    if (opts) o = *opts;
    return h->impl->newton_step(slot, dtau, o, workspace, workspace_bytes, info);
}

int rve_step_dissipation_batch(rve_handle* hs, int count, const double* dtau,
                               rve_step_info* info, int* status) {
    if (!hs || count < 0 || !dtau) return RVE_EINVAL;
    std::vector<int> rcs(count, RVE_OK);
    std::vector<std::thread> th;
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) { rcs[i] = RVE_EINVAL; continue; }
        th.emplace_back([&, i]() { rcs[i] = rve_step_dissipation(hs[i], dtau[i], info ? &info[i] : nullptr); });
    }
    for (auto& t : th) t.join();
    int rc = RVE_OK;
    for (int i = 0; i < count; ++i) {
        if (status) status[i] = rcs[i];
        if (rcs[i] != RVE_OK) rc = rcs[i];
    }
    return rc;
}

int rve_effective_toughness_slot(rve_handle h, int slot, double* G) {
    if (!h || !G || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    if (int rc = h->impl->drop_kept(slot)) return rc;
    const SlotState& s = h->impl->slots[slot];
    if (!s.ready) { h->err = "set_microstructure first"; return RVE_ESTATE; }
    if (!s.fractured) { h->err = "fracture point not reached"; return RVE_ENOTDONE; }
    *G = s.V * (s.T - 0.5 * s.Sigma * s.E) / s.A_g;
    return RVE_OK;
}

int rve_effective_toughness(rve_handle h, double* G) { return rve_effective_toughness_slot(h, 0, G); }

int rve_get_field_slot(rve_handle h, int slot, int which, double* host, size_t count) {
    if (!h || !host) return RVE_EINVAL;
    return h->impl->get_field(slot, which, host, count);
}
int rve_get_field(rve_handle h, int which, double* host, size_t count) {
    return rve_get_field_slot(h, 0, which, host, count);
}
int rve_set_field_slot(rve_handle h, int slot, int which, const double* host, size_t count) {
    if (!h || !host) return RVE_EINVAL;
    return h->impl->set_field(slot, which, host, count);
}
int rve_set_field(rve_handle h, int which, const double* host, size_t count) {
    return rve_set_field_slot(h, 0, which, host, count);
}

int rve_state_bytes(rve_handle h, size_t* bytes) {
    if (!h || !bytes) return RVE_EINVAL;
    *bytes = h->impl->state_bytes();
    return RVE_OK;
}
int rve_save_state(rve_handle h, int slot, void* host, size_t bytes) {
    if (!h || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    return h->impl->save_state(slot, host, bytes);
}
int rve_load_state(rve_handle h, int slot, const void* host, size_t bytes) {
    if (!h || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    return h->impl->load_state(slot, host, bytes);
}

int rve_get_scalars_slot(rve_handle h, int slot, double* o) {
    if (!h || !o || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    if (int rc = h->impl->drop_kept(slot)) return rc;
    const SlotState& s = h->impl->slots[slot];
    o[0] = s.E;
    o[1] = s.Sigma;
    o[2] = s.T;
    o[3] = s.tau;
    o[4] = s.tau0;
    o[5] = s.step;
    o[6] = s.fractured ? 1.0 : 0.0;
    o[7] = s.A_g;
    return RVE_OK;
}
int rve_get_scalars(rve_handle h, double* o) {
    double t[8];
    int rc = rve_get_scalars_slot(h, 0, t);
    if (rc == RVE_OK && o) std::memcpy(o, t, sizeof(double) * 6);
    return rc;
}

int rve_set_scalars_slot(rve_handle h, int slot, const double* in) {
    if (!h || !in || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(in[i])) return RVE_EINVAL;
    if (int rc = h->impl->drop_kept(slot)) return rc;
    SlotState& s = h->impl->slots[slot];
    s.E = in[0];
    s.Sigma = in[1];
    s.T = in[2];
    s.tau = in[3];
    s.tau0 = in[4];
    s.step = (int)in[5];
    return RVE_OK;
}
int rve_set_scalars(rve_handle h, const double* in) { return rve_set_scalars_slot(h, 0, in); }

int rve_release_slot(rve_handle h, int slot) {
    if (!h || slot < 0 || slot >= h->impl->B) return RVE_EINVAL;
    if (int rc = h->impl->drop_kept(slot)) return rc;
    h->impl->slots[slot] = SlotState();
    return RVE_OK;
}

int rve_apply_green_op(rve_handle h, const double* eps, double* out) {
    if (!h || !eps || !out) return RVE_EINVAL;
    return h->impl->apply_green(0, eps, out);
}

int rve_apply_green_op_device(rve_handle h, const void* eps, void* out, int repeat) {
    if (!h || !eps || !out || repeat < 0) return RVE_EINVAL;
    return h->impl->apply_green_device(eps, out, repeat);
}

int rve_apply_green_op_device_noalloc(rve_handle h, const void* eps, void* out, int repeat) {
    if (!h) return RVE_EINVAL;
    if (!eps || !out || repeat < 0) { h->err = "null device pointer or repeat < 0"; return RVE_EINVAL; }
    if (!h->scratch) { h->err = "static scratch array unavailable on this device"; return RVE_EDEVICE; }
    return h->impl->apply_green_device_scratch(h->scratch, RVE_NOALLOC_SCRATCH_BYTES, eps, out, repeat);
}

int rve_solve_mechanics(rve_handle h, int* it, double* Sigma1) {
    if (!h) return RVE_EINVAL;
    return h->impl->solve_mechanics(0, it, Sigma1);
}

int rve_solve_damage(rve_handle h, double E, double* D, int* it, int commit) {
    if (!h || !(E >= 0.0)) return RVE_EINVAL;
    return h->impl->solve_damage(0, E, D, it, commit);
}

int rve_dissipation(rve_handle h, double* D, double* G) {
    if (!h) return RVE_EINVAL;
    return h->impl->dissipation(0, D, G);
}

int rve_autotune(rve_handle h, int repeat, int* shape_out) {
    if (!h) return RVE_EINVAL;
    return h->impl->autotune(repeat, shape_out);
}

int rve_profile_pass(rve_handle h, int pass, int repeat, double* bytes_per_launch) {
    if (!h || repeat < 0) return RVE_EINVAL;
    return h->impl->profile_pass(pass, repeat, bytes_per_launch);
}

const char* rve_last_error(rve_handle h) { return h ? h->err.c_str() : g_last_error.c_str(); }

const char* rve_version(void) { return "mirve 0.2 (gfx950)"; }

}  // extern "C"
