// Internal declarations shared by the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mirve {

constexpr int kMaxStages = 12;     // radix stages per axis (N <= 1024)
constexpr int kMaxMat = 65536;     // material table entries
constexpr int kRedBlocks = 1024;   // max blocks of a reduction kernel

// Keeps the scheduler from sinking the loads above it to their uses below:
// the loads of a round are all in flight before the first use waits.
__device__ __forceinline__ void loads_issued() { __builtin_amdgcn_sched_barrier(0); }

template <typename T>
struct cplx {
    T x, y;
};

template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ inline cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

// Mixed-radix Stockham plan of one axis.  Twiddles w_N^m = exp(-2 pi i m/N),
// m = 0..N-1, live at tw_off (in elements of cplx<T>) of the twiddle table.
struct AxisPlan {
    int N;
    int nst;
    int rad[kMaxStages];
    int tw_off;
    int min_rad;
    int fastN;       // N when the fixed-size two-level FFT is used, else 0
};

// Per-material constants, indexed by the per-voxel material id.  The
// stiffness is the Mandel matrix of the (rotated) phase stiffness, already
// multiplied by k for notch voxels.
template <typename T>
struct MatEntry {
    T C[36];         // s x s Mandel stiffness, row-major, s = 3 or 6
    T K;             // bulk modulus (C:I = 3K I)
    T Gc;            // critical energy release rate
    T drive;         // 1, or 0 on notch voxels (no elastic driving force)
    T pad;
    T A[6];          // cleavage tensor A_f = I + beta (I - n n) (Eq. 15) in the
                     // order xx, yy, zz, yz, xz, xy (2D: xx, yy, xy used)
};

// Geometry shared by all kernels of a handle.
struct Geom {
    int dim, s;
    int nx, ny, nz;
    int nxh;                  // nx / 2 + 1
    long long N;              // voxels
    long long Nspec;          // nxh * ny * nz (complex per component); layout [kx][z][y]
    double h, ell, k_res;
    double inv_N;             // 1 / N (inverse DFT normalisation)
    int B;                    // RVEs in the batch
    int mstride;              // material-table entries per RVE
    int aniso;                // 1 when some phase has a cleavage tensor A != I
};

}  // namespace mirve
