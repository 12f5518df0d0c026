// Device-side views and kernel launchers of the shell multigrid (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mgk {

// The couplings one step of a column sweep needs, in the order a wavefront
// walks its half of the column: record t of direction dir (0: upward from
// layer 0, 1: downward from layer nz-1) and row J is that of layer
// k = dir ? nz-1-t : t (clamped to [0, nz-1]): Tlam[k][J], Tth[k][J],
// Tth[k][J+1], and tc, the vertical coupling to the next layer in that
// direction (Tr[k+1][J] upward, Tr[k][J] downward). Table layout
// [dir][J][t], kStepStride records per row.
template <typename T>
struct alignas(4 * sizeof(T)) StepCoef {
    T tl, ts, tn, tc;
};
constexpr int kStepStride = 72;

// Geometry and operator data of one level, in the precision T of the kernels
// that read it. Fields are [k][J][i] with i fastest; plane = nI*nJ.
template <typename T>
struct LevelView {
    int nI, nJ, nz;
    long long plane;
    const T* Tlam;   // [nz][nJ]
    const T* Tth;    // [nz][nJ+1], face F south of row F
    const T* Tr;     // [nz+1][nJ], face F below layer F
    const T* M;      // [nz][plane] mass sum(alpha V)
    const T* invp;   // [nz][plane] inverse pivots of the twisted factorisation of H_z
    const StepCoef<T>* sc;   // [2][nJ][kStepStride] step records (see StepCoef)
};

// Maps between a fine level and the next coarser one.
template <typename T>
struct TransferView {
    int nIc, nJc;
    const int* crow_of;      // [nJf]   coarse row of each fine row
    const int* prow;         // [2nJf]  latitude rows used by P
    const T* pw;             // [2nJf]  their weights
    const int* child_first;  // [nJc]   first fine row of each coarse row
    const int* child_count;  // [nJc]   1 or 2
    const int* ptrow;        // [4nJc]  fine rows gathered by P^T (-1 unused)
    const T* ptw;            // [4nJc]
};

constexpr int kBlock = 256;

inline int blocks_for(long long n) { return int((n + kBlock - 1) / kBlock); }

// --- launchers (all asynchronous on `s`) ---------------------------------

// y = H x, or y = f - H x when f != nullptr (difference form).
template <typename T>
void apply(const LevelView<T>& L, const T* x, const T* f, T* y, hipStream_t s);

// One damped block-Jacobi sweep (Eq. 1):
//   xout = (1-omega) xin + omega H_z^{-1}(f + sum_h T_h xin_nb),
// or the sweep from zero xout = omega H_z^{-1} f when xin == nullptr.
// Levels with fewer than staged_columns columns use the staged kernel.
template <typename T>
void smooth(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega,
            long long staged_columns, hipStream_t s);

// The same sweep with the kernel for levels that fill the GPU (k_sweep.hip),
// which smooth() uses on every level it does not stage.
template <typename T>
void sweep(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega, hipStream_t s);

// The whole coarsest-level solve in one launch (one block): `sweeps` sweeps
// from zero, ping-ponging between xa and xb. Returns 0 if the result is in
// xa, 1 if in xb. Meant for levels of at most kCoarseSolveColumns columns;
// levels of at most kCoarseLdsColumns columns whose data fit in max_lds bytes
// of LDS (see coarse_lds_bytes) run entirely in LDS.
constexpr long long kCoarseSolveColumns = 4096;
constexpr long long kCoarseLdsColumns = 128;
template <typename T>
int coarse_solve(const LevelView<T>& L, const T* f, T* xa, T* xb, T omega, int sweeps,
                 size_t max_lds, hipStream_t s);

// LDS bytes of the one-block coarsest solve: f, pivots and iterate per cell,
// the three coefficient tables, and the exchange slots of two wavefront
// pairs. unit: the unit-vector solves of coarse_basis, which store no f and
// read the two horizontal tables from global memory.
template <typename T>
inline size_t coarse_lds_bytes(long long plane, int nJ, int nz, bool unit = false) {
    const size_t horiz = unit ? 0 : size_t(nz) * nJ + size_t(nz) * (nJ + 1);
    return ((unit ? 2 : 3) * size_t(plane) * size_t(nz) + horiz + size_t(nz + 1) * nJ + 512) *
           sizeof(T);
}

// The coarsest-level solve (`sweeps` sweeps from zero) is a linear map
// x = C f of the level's n cells. coarse_basis writes C^T, row by row (row j
// is the solve applied to the j-th unit vector), in FP64 into Ct (n*n
// values), with one block per row and the level held in LDS. Returns false,
// launching nothing, if n > kDenseCoarseMax or the level does not fit in
// max_lds bytes of LDS.
constexpr long long kDenseCoarseMax = 6144;
bool coarse_basis(const LevelView<double>& L, double* Ct, double omega, int sweeps,
                  size_t max_lds, hipStream_t s);

// B = A^T for n x n row-major matrices (A and B distinct).
template <typename T>
void transpose_square(const T* A, T* B, long long n, hipStream_t s);

// x = A f for an n x n row-major matrix: one wavefront per row, partial sums
// in a fixed order (results are reproducible).
template <typename T>
void dense_matvec(const T* A, long long n, const T* f, T* x, hipStream_t s);

// fc = R (f - H x) (sum over children), or R f when x == nullptr.
template <typename T>
void restrict_residual(const LevelView<T>& F, const TransferView<T>& X, const T* f,
                       const T* x, T* fc, hipStream_t s);

// x += P xc (bilinear, cell-centred).
template <typename T>
void prolong_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                 hipStream_t s);

// xc = P^T x.
template <typename T>
void prolong_transpose(const LevelView<T>& F, const TransferView<T>& X, const T* x,
                       T* xc, hipStream_t s);

// x += R^T xc (every child cell takes its coarse parent's value).
template <typename T>
void inject_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                hipStream_t s);

// Refinement step on the finest level, in the iterate's precision TU (FP64;
// FP32 in the pure single-precision solve):
//   unew = uin + e (or uin when e == nullptr), written to uout if set;
//   r = b - H unew, stored as TR; per-block partial sums of r^2 in FP64,
//   and of b^2 into partials_b when it is not null.
// uin == nullptr stands for a zero iterate (a solve from u = 0): it is not
// read, and with e == nullptr as well the step is r = b.
// Returns the number of blocks (partials written): at most
// max(residual_update_blocks(L), blocks_for(L.plane)).
template <typename TU, typename TE, typename TR>
int residual_update(const LevelView<TU>& L, const TU* b, const TU* uin, const TE* e, TU* uout,
                    TR* r, double* partials, double* partials_b, hipStream_t s);
// Blocks (hence partial sums) residual_update launches for level L.
template <typename TU>
int residual_update_blocks(const LevelView<TU>& L);

// out[c] = sum of partials[c*stride + 0..n) in a fixed order, c < count.
void sum_partials(const double* partials, int n, double* out, hipStream_t s, int count = 1,
                  long long stride = 0);

// Setup: M = alpha * V (fine level; not written when M is null) and
// per-block counts of alpha values that are not finite and > 0 (as FP64
// partials).
int fine_mass(const LevelView<double>& L, const double* V, const double* alpha,
              double* M, double* partials, hipStream_t s);
// Setup: row-sum pivots of the twisted factorisation of H_z (eliminated from
// both ends toward layer nz/2); inverse pivots in FP64 and FP32 and an FP32
// copy of M.
void pivots(const LevelView<double>& L, double* invp64, float* invp32, float* M32,
            hipStream_t s);

void grad_alpha(const LevelView<double>& L, const double* V, const double* lam,
                const double* u, double* g, hipStream_t s);
void cell_volumes(const LevelView<double>& L, const double* V, double* out, hipStream_t s);
template <typename TA, typename TB>
void cast(const TA* in, TB* out, long long n, hipStream_t s);
template <typename T>
void fill(T* out, T v, long long n, hipStream_t s);

}  // namespace mgk
