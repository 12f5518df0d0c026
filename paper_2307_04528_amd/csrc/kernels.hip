// HIP kernels of the shell multigrid for gfx950 (CDNA4).
//
// Mapping. Kernels that walk a vertical column (the Thomas solves, and every
// stencil, which needs the layers above and below) use one lane per column
// (I, J); a wavefront covers 64 consecutive longitudes of a row, so every
// layer k is one coalesced 256 B (FP32) / 512 B (FP64) access per wavefront.
// Kernels with no vertical coupling (prolongation, its transpose, gradient)
// use one lane per cell.
//
// Latency. A column kernel is a chain of nz dependent steps; to keep many
// loads in flight per lane, the layer loop is fully unrolled over a
// compile-time bucket NZ >= nz and every load is unconditional: layer indices
// are clamped to nz-1, neighbour offsets at the poles are clamped to the cell
// itself (their coefficient in the tables is exactly 0), and the top/bottom
// vertical coefficients are 0. Only stores are guarded. Thomas forward values
// stay in registers. The Thomas sweeps prefetch explicitly: the loads of the
// next chunk of layers are issued before the current chunk is solved, with
// scheduling barriers so the compiler neither serialises them nor hoists
// everything (which would spill). Each layer of a per-cell array is addressed
// as a wave-uniform base (scalar registers) plus a 32-bit per-lane offset.
//
// L2 locality. The hardware hands block b to XCD b % 8; blocks are remapped
// so each XCD works on one contiguous range of columns, so the latitude
// neighbours a stencil re-reads come from the same L2.
#include "kernels.hpp"

#include <cstdint>
#include <type_traits>

namespace mgk {

namespace {

__device__ __forceinline__ long long logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
    return (long long)(x * q + (x < r ? x : r) + s);
}

__device__ __forceinline__ long long column_index() {
    return logical_block() * blockDim.x + threadIdx.x;
}

// Offsets of the four horizontal neighbours of a column; at a pole the
// neighbour offset is 0 (the cell itself) and the face coefficient is 0.
struct Col {
    int J, i;
    long long dw, de, ds, dn;
};

__device__ __forceinline__ Col locate(long long col, int nI, int nJ) {
    Col c;
    c.J = int(col / nI);
    c.i = int(col - (long long)c.J * nI);
    c.dw = (c.i == 0) ? nI - 1 : -1;
    c.de = (c.i == nI - 1) ? -(nI - 1) : 1;
    c.ds = (c.J > 0) ? -nI : 0;
    c.dn = (c.J < nJ - 1) ? nI : 0;
    return c;
}

__device__ __forceinline__ int clampk(int k, int nz) { return k < nz ? k : nz - 1; }

__device__ __forceinline__ uint32_t column_index32() {
    return uint32_t(logical_block()) * blockDim.x + threadIdx.x;
}

// Element offsets (within one layer) of a column and of its four horizontal
// neighbours, as 32-bit values: every layer is then addressed as a
// wave-uniform base pointer plus these offsets. At a pole the missing
// neighbour is the cell itself (its face coefficient is 0). ROWU: every
// wavefront lies inside one latitude row (nI a multiple of 64), so the row
// index -- and every coefficient-table address -- is wave-uniform.
struct Nb {
    uint32_t c, w, e, s, n;
    int J;
};

template <bool ROWU>
__device__ __forceinline__ Nb neighbours(uint32_t col, int nI, int nJ) {
    int J = int(col / uint32_t(nI));
    if constexpr (ROWU) J = __builtin_amdgcn_readfirstlane(J);
    const int i = int(col) - J * nI;
    Nb b;
    b.J = J;
    b.c = col;
    b.w = (i == 0) ? col + uint32_t(nI - 1) : col - 1u;
    b.e = (i == nI - 1) ? col - uint32_t(nI - 1) : col + 1u;
    b.s = (J > 0) ? col - uint32_t(nI) : col;
    b.n = (J < nJ - 1) ? col + uint32_t(nI) : col;
    return b;
}

// The same offsets in bytes for element type T (a layer of any per-cell
// array is < 4 GiB), so that a load is base(layer, uniform) + 32-bit offset.
template <typename T>
struct NbB {
    uint32_t c, w, e, s, n;
    int J;
    __device__ __forceinline__ explicit NbB(const Nb& b)
        : c(b.c * uint32_t(sizeof(T))), w(b.w * uint32_t(sizeof(T))),
          e(b.e * uint32_t(sizeof(T))), s(b.s * uint32_t(sizeof(T))),
          n(b.n * uint32_t(sizeof(T))), J(b.J) {}
};

// Wave-uniform base of layer kk of a per-cell array (layer stride Pb bytes),
// pinned to scalar registers so that every access is issued as a global load
// or store with a scalar base and a 32-bit per-lane byte offset.
__device__ __forceinline__ uint64_t uniform64(uint64_t p) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(p));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(p >> 32));
    return (uint64_t(hi) << 32) | lo;
}
typedef const __attribute__((address_space(1))) char* gcptr;   // global memory
typedef __attribute__((address_space(1))) char* gptr;

template <typename T>
__device__ __forceinline__ gcptr layer(const T* a, int kk, uint64_t Pb) {
    return (gcptr)(uniform64(reinterpret_cast<uint64_t>(a) + uint64_t(kk) * Pb));
}
template <typename T>
__device__ __forceinline__ gptr layer_w(T* a, int kk, uint64_t Pb) {
    return (gptr)(uniform64(reinterpret_cast<uint64_t>(a) + uint64_t(kk) * Pb));
}
template <typename T>
__device__ __forceinline__ T ldb(gcptr base, uint32_t boff) {
    return *(const __attribute__((address_space(1))) T*)(base + boff);
}
template <typename T>
__device__ __forceinline__ void stb(gptr base, uint32_t boff, T v) {
    *(__attribute__((address_space(1))) T*)(base + boff) = v;
}

// Read-only coefficient tables through the constant address space: with a
// wave-uniform index this is a scalar load.
template <typename T>
__device__ __forceinline__ T tab(const T* p, int idx) {
    return ((const __attribute__((address_space(4))) T*)p)[idx];
}

template <typename T>
__device__ __forceinline__ void block_sum_to(T v, T* out) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __shared__ T red[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) t += red[w];
        *out = t;
    }
}

// Horizontal part of H at one cell in difference form (coefficients already
// loaded): Tlam (2xc - xw - xe) + Ts (xc - xs) + Tn (xc - xn).
template <typename T>
__device__ __forceinline__ T hdiff(T tl, T ts, T tn, T xc, T xw, T xe, T xs, T xn) {
    return tl * ((xc - xw) + (xc - xe)) + ts * (xc - xs) + tn * (xc - xn);
}

// ---------------------------------------------------------------------------
// y = H x (HAS_F = false) or y = f - H x (HAS_F = true)
template <typename T, int NZ, bool HAS_F>
__global__ __launch_bounds__(kBlock) void k_apply(LevelView<T> L, const T* __restrict__ x,
                                                  const T* __restrict__ f,
                                                  T* __restrict__ y) {
    const long long col = column_index();
    if (col >= L.plane) return;
    const Col c = locate(col, L.nI, L.nJ);
    const int nJ = L.nJ, nz = L.nz;
    const long long P = L.plane;
    const T* xc0 = x + col;
    T xm = 0, xcur = xc0[0];
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
        const long long o = kk * P;
        const T xp = xc0[kp * P];
        T h = L.M[col + o] * xcur +
              hdiff(L.Tlam[kk * nJ + c.J], L.Tth[kk * (nJ + 1) + c.J],
                    L.Tth[kk * (nJ + 1) + c.J + 1], xcur, xc0[o + c.dw], xc0[o + c.de],
                    xc0[o + c.ds], xc0[o + c.dn]) +
              L.Tr[kk * nJ + c.J] * (xcur - xm) + L.Tr[(kk + 1) * nJ + c.J] * (xcur - xp);
        if (k < nz) y[col + o] = HAS_F ? f[col + o] - h : h;
        xm = xcur;
        xcur = xp;
    }
}

// ---------------------------------------------------------------------------
// Block-Jacobi sweep (Eq. 1):
//   xout = (1-omega) xin + omega H_z^{-1}(f + sum_h T_h xin_nb)   (HAS_X)
//   xout = omega H_z^{-1} f                                       (!HAS_X)
//
// Register budget: the Thomas forward values y[NZ] live in registers; the
// occupancy target (waves per SIMD) caps how far ahead the compiler may hoist
// the next layers' loads. KEEP_P also keeps the inverse pivots (else the
// backward sweep re-reads them, mostly from cache).
#ifndef MG_SMOOTH_KEEP_P
#define MG_SMOOTH_KEEP_P 0
#endif
#ifndef MG_SMOOTH_WAVES32
#define MG_SMOOTH_WAVES32 2
#endif
#ifndef MG_SMOOTH_WAVES64
#define MG_SMOOTH_WAVES64 1
#endif
#ifndef MG_CHUNK32
#define MG_CHUNK32 4
#endif
#ifndef MG_CHUNK64
#define MG_CHUNK64 4
#endif
template <typename T>
struct ColumnWaves {
    static constexpr int value = std::is_same<T, float>::value ? MG_SMOOTH_WAVES32
                                                                : MG_SMOOTH_WAVES64;
};
// Layers per prefetch chunk: the loads of chunk c+1 are issued before chunk
// c is solved (scheduling barriers keep the compiler from hoisting further).
template <typename T>
struct ChunkDepth {
    static constexpr int value = std::is_same<T, float>::value ? MG_CHUNK32 : MG_CHUNK64;
};

template <typename T, int NZ, bool KEEP_P, bool HAS_X, bool ROWU>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ColumnWaves<T>::value)))
void k_smooth(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ xin,
              T* __restrict__ xout, T omega) {
    const uint32_t col = column_index32();
    if (col >= uint32_t(L.plane)) return;
    const NbB<T> b(neighbours<ROWU>(col, L.nI, L.nJ));
    const int nJ = L.nJ, nz = L.nz;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    constexpr int D = ChunkDepth<T>::value;
    constexpr int NC = (NZ + D - 1) / D;
    T y[NC * D];
    T ip[KEEP_P ? NC * D : 1];
    // double-buffered chunk of D layers: right-hand side and inverse pivot
    T bs[2][D], bp[2][D];
    auto load = [&](int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kk = clampk(c * D + d, nz);
            T s = ldb<T>(layer(f, kk, Pb), b.c);
            if constexpr (HAS_X) {
                gcptr xk = layer(xin, kk, Pb);
                s += tab(L.Tlam, kk * nJ + b.J) * (ldb<T>(xk, b.w) + ldb<T>(xk, b.e)) +
                     tab(L.Tth, kk * (nJ + 1) + b.J) * ldb<T>(xk, b.s) +
                     tab(L.Tth, kk * (nJ + 1) + b.J + 1) * ldb<T>(xk, b.n);
            }
            bs[buf][d] = s;
            bp[buf][d] = ldb<T>(layer(L.invp, kk, Pb), b.c);
        }
    };
    T yp = 0;
    load(0, 0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c + 1 < NC) load(c + 1, (c + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kk = clampk(c * D + d, nz);
            yp = (bs[c & 1][d] + tab(L.Tr, kk * nJ + b.J) * yp) * bp[c & 1][d];
            y[c * D + d] = yp;
            if constexpr (KEEP_P) ip[c * D + d] = bp[c & 1][d];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // backward substitution, top layer first, with the same chunked prefetch
    // of the inverse pivots and of the old iterate
    T bq[2][D], bx[2][D];
    auto load_back = [&](int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kk = clampk(c * D + d, nz);
            if constexpr (!KEEP_P) bq[buf][d] = ldb<T>(layer(L.invp, kk, Pb), b.c);
            if constexpr (HAS_X) bx[buf][d] = ldb<T>(layer(xin, kk, Pb), b.c);
        }
    };
    T xn = 0;
    const T keep = T(1) - omega;
    load_back(NC - 1, (NC - 1) & 1);
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
        if (c > 0) load_back(c - 1, (c - 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int k = c * D + d;
            const int kk = clampk(k, nz);
            T p;
            if constexpr (KEEP_P) p = ip[k]; else p = bq[c & 1][d];
            xn = (k < nz) ? y[k] + tab(L.Tr, (kk + 1) * nJ + b.J) * p * xn : T(0);
            T out = omega * xn;
            if constexpr (HAS_X) out += keep * bx[c & 1][d];
            if (k < nz) stb<T>(layer_w(xout, kk, Pb), b.c, out);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// One lane per coarse column: sum of (f - H x) over its 2 x (1 or 2) children.
// Children rows j0, j1 (j1 = j0 when the row is not merged, weight 0).
template <typename T, int NZ, bool HAS_X>
__global__ __launch_bounds__(kBlock) void k_restrict_residual(LevelView<T> F, TransferView<T> X,
                                                              const T* __restrict__ f,
                                                              const T* __restrict__ x,
                                                              T* __restrict__ fc) {
    const long long colc = column_index();
    const long long Pc = (long long)X.nIc * X.nJc;
    if (colc >= Pc) return;
    const int nI = F.nI, nJ = F.nJ, nz = F.nz;
    const long long P = F.plane;
    const int Jc = int(colc / X.nIc);
    const int Ic = int(colc - (long long)Jc * X.nIc);
    const int j0 = X.child_first[Jc];
    const int two = X.child_count[Jc] - 1;           // 0 or 1
    const int j1 = j0 + two;
    const T w1 = T(two);
    const int i0 = 2 * Ic, i1 = i0 + 1;
    const int iw = (i0 == 0) ? nI - 1 : i0 - 1;
    const int ie = (i1 == nI - 1) ? 0 : i1 + 1;
    const long long r0 = (long long)j0 * nI, r1 = (long long)j1 * nI;
    const long long rs = (j0 > 0) ? r0 - nI : r0;    // south of j0 (coefficient 0 at a pole)
    const long long rn = (j1 < nJ - 1) ? r1 + nI : r1;
    // vertical window of the four children
    T m00 = 0, m01 = 0, m10 = 0, m11 = 0;
    T c00 = 0, c01 = 0, c10 = 0, c11 = 0;
    if constexpr (HAS_X) {
        c00 = x[r0 + i0]; c01 = x[r0 + i1]; c10 = x[r1 + i0]; c11 = x[r1 + i1];
    }
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
        const long long o = kk * P;
        T acc = f[o + r0 + i0] + f[o + r0 + i1] + w1 * (f[o + r1 + i0] + f[o + r1 + i1]);
        if constexpr (HAS_X) {
            const long long op = kp * P;
            const T p00 = x[op + r0 + i0], p01 = x[op + r0 + i1];
            const T p10 = x[op + r1 + i0], p11 = x[op + r1 + i1];
            const T tl0 = F.Tlam[kk * nJ + j0], tl1 = F.Tlam[kk * nJ + j1];
            const T ts0 = F.Tth[kk * (nJ + 1) + j0], tn0 = F.Tth[kk * (nJ + 1) + j0 + 1];
            const T ts1 = F.Tth[kk * (nJ + 1) + j1], tn1 = F.Tth[kk * (nJ + 1) + j1 + 1];
            const T tb0 = F.Tr[kk * nJ + j0], tt0 = F.Tr[(kk + 1) * nJ + j0];
            const T tb1 = F.Tr[kk * nJ + j1], tt1 = F.Tr[(kk + 1) * nJ + j1];
            const T xw0 = x[o + r0 + iw], xe0 = x[o + r0 + ie];
            const T xw1 = x[o + r1 + iw], xe1 = x[o + r1 + ie];
            const T xs0 = x[o + rs + i0], xs1 = x[o + rs + i1];
            const T xn0 = x[o + rn + i0], xn1 = x[o + rn + i1];
            // row j0: north neighbour is row j1 when merged, else rn
            const T n00 = two ? c10 : xn0, n01 = two ? c11 : xn1;
            // row j1: south neighbour is row j0 when merged, else rs
            const T s10 = two ? c00 : xs0, s11 = two ? c01 : xs1;
            T h0 = F.M[o + r0 + i0] * c00 + hdiff(tl0, ts0, tn0, c00, xw0, c01, xs0, n00) +
                   F.M[o + r0 + i1] * c01 + hdiff(tl0, ts0, tn0, c01, c00, xe0, xs1, n01) +
                   tb0 * ((c00 - m00) + (c01 - m01)) + tt0 * ((c00 - p00) + (c01 - p01));
            T h1 = F.M[o + r1 + i0] * c10 + hdiff(tl1, ts1, tn1, c10, xw1, c11, s10, xn0) +
                   F.M[o + r1 + i1] * c11 + hdiff(tl1, ts1, tn1, c11, c10, xe1, s11, xn1) +
                   tb1 * ((c10 - m10) + (c11 - m11)) + tt1 * ((c10 - p10) + (c11 - p11));
            acc -= h0 + w1 * h1;
            m00 = c00; m01 = c01; m10 = c10; m11 = c11;
            c00 = p00; c01 = p01; c10 = p10; c11 = p11;
        }
        if (k < nz) fc[kk * Pc + colc] = acc;
    }
}

// ---------------------------------------------------------------------------
// x += P xc, one lane per fine cell: bilinear interpolation (3/4, 1/4 in
// longitude; the row weights of the map in latitude).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView<T> F, TransferView<T> X,
                                                        const T* __restrict__ xc,
                                                        T* __restrict__ x, long long n) {
    const long long t = logical_block() * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const long long P = F.plane;
    const int k = int(t / P);
    const long long col = t - k * P;
    const int j = int(col / F.nI);
    const int i = int(col - (long long)j * F.nI);
    const int nIc = X.nIc;
    const int J0 = X.prow[2 * j], J1 = X.prow[2 * j + 1];
    const T w0 = X.pw[2 * j], w1 = X.pw[2 * j + 1];
    const int I = i >> 1;
    const int In = (i & 1) ? (I + 1 == nIc ? 0 : I + 1) : (I == 0 ? nIc - 1 : I - 1);
    const T* lay = xc + (long long)k * nIc * X.nJc;
    const T* c0 = lay + (long long)J0 * nIc;
    const T* c1 = lay + (long long)J1 * nIc;
    const T a = T(0.75), b = T(0.25);
    x[t] += w0 * (a * c0[I] + b * c0[In]) + w1 * (a * c1[I] + b * c1[In]);
}

// xc = P^T x, one lane per coarse cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_T(LevelView<T> F, TransferView<T> X,
                                                      const T* __restrict__ x,
                                                      T* __restrict__ xc, long long nc) {
    const long long t = logical_block() * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    const long long Pc = (long long)X.nIc * X.nJc;
    const int k = int(t / Pc);
    const long long colc = t - k * Pc;
    const int Jc = int(colc / X.nIc);
    const int Ic = int(colc - (long long)Jc * X.nIc);
    const int nIf = F.nI;
    const int iE = 2 * Ic, iO = 2 * Ic + 1;
    const int iW = (iE == 0) ? nIf - 1 : iE - 1;
    const int iEE = (iO + 1 == nIf) ? 0 : iO + 1;
    const T a = T(0.75), b = T(0.25);
    T acc = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = X.ptrow[4 * Jc + e];
        const T w = X.ptw[4 * Jc + e];
        const T* r = x + k * F.plane + (long long)(row < 0 ? 0 : row) * nIf;
        acc += w * (a * (r[iE] + r[iO]) + b * (r[iW] + r[iEE]));
    }
    xc[t] = acc;
}

// fb += y, xb -= H y with y = R^T fcb (every child takes its coarse value).
template <typename T, int NZ>
__global__ __launch_bounds__(kBlock) void k_inject_residual_adj(LevelView<T> F,
                                                                TransferView<T> X,
                                                                const T* __restrict__ fcb,
                                                                T* __restrict__ xb,
                                                                T* __restrict__ fb) {
    const long long col = column_index();
    if (col >= F.plane) return;
    const int nI = F.nI, nJ = F.nJ, nz = F.nz, nIc = X.nIc;
    const int j = int(col / nI);
    const int i = int(col - (long long)j * nI);
    const long long Pc = (long long)nIc * X.nJc;
    const int iw = (i == 0) ? nI - 1 : i - 1, ie = (i == nI - 1) ? 0 : i + 1;
    const long long oc = (long long)X.crow_of[j] * nIc;
    const long long cc = oc + (i >> 1), cw = oc + (iw >> 1), ce = oc + (ie >> 1);
    const long long cs = (j > 0) ? (long long)X.crow_of[j - 1] * nIc + (i >> 1) : cc;
    const long long cn = (j < nJ - 1) ? (long long)X.crow_of[j + 1] * nIc + (i >> 1) : cc;
    T ym = 0, yc = fcb[cc];
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
        const T* lay = fcb + kk * Pc;
        const T yp = fcb[kp * Pc + cc];
        const long long o = kk * F.plane + col;
        const T h = F.M[o] * yc +
                    hdiff(F.Tlam[kk * nJ + j], F.Tth[kk * (nJ + 1) + j],
                          F.Tth[kk * (nJ + 1) + j + 1], yc, lay[cw], lay[ce], lay[cs], lay[cn]) +
                    F.Tr[kk * nJ + j] * (yc - ym) + F.Tr[(kk + 1) * nJ + j] * (yc - yp);
        const T fo = fb[o] + yc, xo = xb[o] - h;
        if (k < nz) {
            fb[o] = fo;
            xb[o] = xo;
        }
        ym = yc;
        yc = yp;
    }
}

// ---------------------------------------------------------------------------
// Transposed smoother chain kernel (see smooth_transpose in kernels.hpp).
template <typename T, int NZ, bool HAS_Z, bool ACC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ColumnWaves<T>::value)))
void k_smooth_T(LevelView<T> L, const T* xb,
                                                     const T* __restrict__ zin,
                                                     T* xbout,  // may alias xb
                                                     T* __restrict__ zout,
                                                     T* __restrict__ fb, T omega) {
    const long long col = column_index();
    if (col >= L.plane) return;
    const Col c = locate(col, L.nI, L.nJ);
    const int nJ = L.nJ, nz = L.nz;
    const long long P = L.plane;
    const T keep = T(1) - omega;
    const T* zc = zin + col;
    const T* pc = L.invp + col;
    T y[NZ];
    T yp = 0;
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz);
        const long long o = kk * P;
        T s = xb[col + o];
        if constexpr (HAS_Z) {
            const T h = L.Tlam[kk * nJ + c.J] * (zc[o + c.dw] + zc[o + c.de]) +
                        L.Tth[kk * (nJ + 1) + c.J] * zc[o + c.ds] +
                        L.Tth[kk * (nJ + 1) + c.J + 1] * zc[o + c.dn];
            s = keep * s + omega * h;
            if (k < nz) xbout[col + o] = s;
        }
        yp = (s + L.Tr[kk * nJ + c.J] * yp) * pc[o];
        y[k] = yp;
    }
    T zn = 0;
#pragma unroll
    for (int k = NZ - 1; k >= 0; --k) {
        const int kk = clampk(k, nz);
        const long long o = kk * P;
        zn = (k < nz) ? y[k] + L.Tr[(kk + 1) * nJ + c.J] * pc[o] * zn : T(0);
        T fo = omega * zn;
        if constexpr (ACC) fo += fb[col + o];
        if (k < nz) {
            if (zout) zout[col + o] = zn;
            fb[col + o] = fo;
        }
    }
}

template <typename T, int NZ>
__global__ __launch_bounds__(kBlock) void k_adjoint_stencil(LevelView<T> L,
                                                            const T* __restrict__ z,
                                                            T* __restrict__ xb, T omega) {
    const long long col = column_index();
    if (col >= L.plane) return;
    const Col c = locate(col, L.nI, L.nJ);
    const int nJ = L.nJ, nz = L.nz;
    const T keep = T(1) - omega;
    const T* zc = z + col;
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz);
        const long long o = kk * L.plane;
        const T h = L.Tlam[kk * nJ + c.J] * (zc[o + c.dw] + zc[o + c.de]) +
                    L.Tth[kk * (nJ + 1) + c.J] * zc[o + c.ds] +
                    L.Tth[kk * (nJ + 1) + c.J + 1] * zc[o + c.dn];
        const T v = keep * xb[col + o] + omega * h;
        if (k < nz) xb[col + o] = v;
    }
}

// ---------------------------------------------------------------------------
// FP64 update + residual + norm partials (the refinement step).
template <typename TE, typename TR, int NZ, bool HAS_E>
__global__ __launch_bounds__(kBlock) void k_residual_update(
    LevelView<double> L, const double* __restrict__ b, const double* __restrict__ uin,
    const TE* __restrict__ e, double* __restrict__ uout, TR* __restrict__ r,
    double* __restrict__ partials) {
    const long long col = column_index();
    double acc = 0;
    if (col < L.plane) {
        const Col c = locate(col, L.nI, L.nJ);
        const int nJ = L.nJ, nz = L.nz;
        const long long P = L.plane;
        const double* uc0 = uin + col;
        const TE* ec0 = e + col;
        auto un = [&](long long o) -> double {
            double v = uc0[o];
            if constexpr (HAS_E) v += double(ec0[o]);
            return v;
        };
        double um = 0, uc = un(0);
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
            const long long o = kk * P;
            const double up = un(kp * P);
            const double h =
                L.M[col + o] * uc +
                hdiff(L.Tlam[kk * nJ + c.J], L.Tth[kk * (nJ + 1) + c.J],
                      L.Tth[kk * (nJ + 1) + c.J + 1], uc, un(o + c.dw), un(o + c.de),
                      un(o + c.ds), un(o + c.dn)) +
                L.Tr[kk * nJ + c.J] * (uc - um) + L.Tr[(kk + 1) * nJ + c.J] * (uc - up);
            const double rv = b[col + o] - h;
            if (k < nz) {
                if constexpr (HAS_E) uout[col + o] = uc;
                r[col + o] = TR(rv);
                acc += rv * rv;
            }
            um = uc;
            uc = up;
        }
    }
    block_sum_to(acc, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_norm2_partials(const double* __restrict__ x,
                                                           long long n,
                                                           double* __restrict__ partials) {
    double acc = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        acc += x[t] * x[t];
    block_sum_to(acc, partials + blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ p, int n,
                                                       double* __restrict__ out) {
    __shared__ double red[1024];
    double acc = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) acc += p[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Setup kernels (FP64).
__global__ __launch_bounds__(kBlock) void k_fine_mass(LevelView<double> L,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ alpha,
                                                      double* __restrict__ M, long long n,
                                                      double* __restrict__ partials) {
    double bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int k = int(t / L.plane);
        const int J = int((t - k * L.plane) / L.nI);
        const double a = alpha[t];
        if (!(a > 0.0) || !isfinite(a)) bad += 1.0;
        M[t] = a * V[k * L.nJ + J];
    }
    block_sum_to(bad, partials + blockIdx.x);
}

// Row-sum form of the Thomas pivots of H_z, per column:
//   mt_k = M_k + 2 Tlam + Tth(south) + Tth(north)
//   g_0 = mt_0, g_k = mt_k + Tr_k g_{k-1} / (Tr_k + g_{k-1}),  p_k = Tr_{k+1} + g_k.
__global__ __launch_bounds__(kBlock) void k_pivots(LevelView<double> L,
                                                   double* __restrict__ invp64,
                                                   float* __restrict__ invp32,
                                                   float* __restrict__ M32) {
    const long long col = column_index();
    if (col >= L.plane) return;
    const int J = int(col / L.nI), nJ = L.nJ;
    double g = 0;
    for (int k = 0; k < L.nz; ++k) {
        const long long o = k * L.plane + col;
        const double mt = L.M[o] + 2.0 * L.Tlam[k * nJ + J] + L.Tth[k * (nJ + 1) + J] +
                          L.Tth[k * (nJ + 1) + J + 1];
        const double trb = L.Tr[k * nJ + J];
        g = (k == 0) ? mt : mt + trb * g / (trb + g);
        const double ip = 1.0 / (L.Tr[(k + 1) * nJ + J] + g);
        invp64[o] = ip;
        invp32[o] = float(ip);
        M32[o] = float(L.M[o]);
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_alpha(LevelView<double> L,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ u,
                                                       double* __restrict__ g, long long n) {
    const long long t = logical_block() * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int k = int(t / L.plane);
    const int J = int((t - k * L.plane) / L.nI);
    g[t] = -lam[t] * V[k * L.nJ + J] * u[t];
}

__global__ __launch_bounds__(kBlock) void k_cell_volumes(LevelView<double> L,
                                                         const double* __restrict__ V,
                                                         double* __restrict__ out,
                                                         long long n) {
    const long long t = logical_block() * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int k = int(t / L.plane);
    const int J = int((t - k * L.plane) / L.nI);
    out[t] = V[k * L.nJ + J];
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kBlock) void k_cast(const TA* __restrict__ in, TB* __restrict__ out,
                                                 long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        out[t] = TB(in[t]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ out, T v, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        out[t] = v;
}

inline int grid_stride_blocks(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    return int(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// Dispatch the layer-count bucket NZ >= nz at compile time.
template <typename F>
void with_nz(int nz, F&& fn) {
    if (nz <= 8) fn(std::integral_constant<int, 8>{});
    else if (nz <= 16) fn(std::integral_constant<int, 16>{});
    else if (nz <= 32) fn(std::integral_constant<int, 32>{});
    else if (nz <= 72) fn(std::integral_constant<int, 72>{});
    else fn(std::integral_constant<int, 128>{});
}

}  // namespace

// --- launchers ---------------------------------------------------------------
template <typename T>
void apply(const LevelView<T>& L, const T* x, const T* f, T* y, hipStream_t s) {
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        if (f) k_apply<T, NZ, true><<<blocks_for(L.plane), kBlock, 0, s>>>(L, x, f, y);
        else k_apply<T, NZ, false><<<blocks_for(L.plane), kBlock, 0, s>>>(L, x, f, y);
    });
}

template <typename T>
void smooth(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega,
            hipStream_t s) {
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        // the backward sweep re-reads the inverse pivots unless KEEP_P
        constexpr bool keep = MG_SMOOTH_KEEP_P != 0;
        const int nb = blocks_for(L.plane);
        if (L.nI % 64 == 0) {
            if (xin) k_smooth<T, NZ, keep, true, true><<<nb, kBlock, 0, s>>>(L, f, xin, xout, omega);
            else k_smooth<T, NZ, keep, false, true><<<nb, kBlock, 0, s>>>(L, f, xin, xout, omega);
        } else {
            if (xin) k_smooth<T, NZ, keep, true, false><<<nb, kBlock, 0, s>>>(L, f, xin, xout, omega);
            else k_smooth<T, NZ, keep, false, false><<<nb, kBlock, 0, s>>>(L, f, xin, xout, omega);
        }
    });
}

template <typename T>
void restrict_residual(const LevelView<T>& F, const TransferView<T>& X, const T* f,
                       const T* x, T* fc, hipStream_t s) {
    const int nb = blocks_for((long long)X.nIc * X.nJc);
    with_nz(F.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        if (x) k_restrict_residual<T, NZ, true><<<nb, kBlock, 0, s>>>(F, X, f, x, fc);
        else k_restrict_residual<T, NZ, false><<<nb, kBlock, 0, s>>>(F, X, f, x, fc);
    });
}

template <typename T>
void prolong_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                 hipStream_t s) {
    const long long n = F.plane * F.nz;
    k_prolong_add<T><<<blocks_for(n), kBlock, 0, s>>>(F, X, xc, x, n);
}

template <typename T>
void prolong_transpose(const LevelView<T>& F, const TransferView<T>& X, const T* x, T* xc,
                       hipStream_t s) {
    const long long nc = (long long)X.nIc * X.nJc * F.nz;
    k_prolong_T<T><<<blocks_for(nc), kBlock, 0, s>>>(F, X, x, xc, nc);
}

template <typename T>
void inject_residual_adjoint(const LevelView<T>& F, const TransferView<T>& X, const T* fcb,
                             T* xb, T* fb, hipStream_t s) {
    with_nz(F.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        k_inject_residual_adj<T, NZ><<<blocks_for(F.plane), kBlock, 0, s>>>(F, X, fcb, xb, fb);
    });
}

template <typename T>
void smooth_transpose(const LevelView<T>& L, const T* xb, const T* zin, T* xbout, T* zout,
                      T* fb, T omega, bool accumulate, hipStream_t s) {
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        const int nb = blocks_for(L.plane);
        if (zin) {
            if (accumulate)
                k_smooth_T<T, NZ, true, true><<<nb, kBlock, 0, s>>>(L, xb, zin, xbout, zout, fb, omega);
            else
                k_smooth_T<T, NZ, true, false><<<nb, kBlock, 0, s>>>(L, xb, zin, xbout, zout, fb, omega);
        } else {
            if (accumulate)
                k_smooth_T<T, NZ, false, true><<<nb, kBlock, 0, s>>>(L, xb, zin, xbout, zout, fb, omega);
            else
                k_smooth_T<T, NZ, false, false><<<nb, kBlock, 0, s>>>(L, xb, zin, xbout, zout, fb, omega);
        }
    });
}

template <typename T>
void adjoint_stencil(const LevelView<T>& L, const T* z, T* xb, T omega, hipStream_t s) {
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        k_adjoint_stencil<T, NZ><<<blocks_for(L.plane), kBlock, 0, s>>>(L, z, xb, omega);
    });
}

template <typename TE, typename TR>
int residual_update(const LevelView<double>& L, const double* b, const double* uin,
                    const TE* e, double* uout, TR* r, double* partials, hipStream_t s) {
    const int nb = blocks_for(L.plane);
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        if (e)
            k_residual_update<TE, TR, NZ, true><<<nb, kBlock, 0, s>>>(L, b, uin, e, uout, r, partials);
        else
            k_residual_update<TE, TR, NZ, false><<<nb, kBlock, 0, s>>>(L, b, uin, e, uout, r, partials);
    });
    return nb;
}

int norm2_partials(const double* x, long long n, double* partials, hipStream_t s) {
    const int nb = grid_stride_blocks(n);
    k_norm2_partials<<<nb, kBlock, 0, s>>>(x, n, partials);
    return nb;
}

void sum_partials(const double* partials, int n, double* out, hipStream_t s) {
    k_sum_partials<<<1, 1024, 0, s>>>(partials, n, out);
}

int fine_mass(const LevelView<double>& L, const double* V, const double* alpha, double* M,
              double* partials, hipStream_t s) {
    const long long n = L.plane * L.nz;
    const int nb = grid_stride_blocks(n);
    k_fine_mass<<<nb, kBlock, 0, s>>>(L, V, alpha, M, n, partials);
    return nb;
}

void pivots(const LevelView<double>& L, double* invp64, float* invp32, float* M32,
            hipStream_t s) {
    k_pivots<<<blocks_for(L.plane), kBlock, 0, s>>>(L, invp64, invp32, M32);
}

void grad_alpha(const LevelView<double>& L, const double* V, const double* lam,
                const double* u, double* g, hipStream_t s) {
    const long long n = L.plane * L.nz;
    k_grad_alpha<<<blocks_for(n), kBlock, 0, s>>>(L, V, lam, u, g, n);
}

void cell_volumes(const LevelView<double>& L, const double* V, double* out, hipStream_t s) {
    const long long n = L.plane * L.nz;
    k_cell_volumes<<<blocks_for(n), kBlock, 0, s>>>(L, V, out, n);
}

template <typename TA, typename TB>
void cast(const TA* in, TB* out, long long n, hipStream_t s) {
    k_cast<TA, TB><<<grid_stride_blocks(n), kBlock, 0, s>>>(in, out, n);
}

template <typename T>
void fill(T* out, T v, long long n, hipStream_t s) {
    k_fill<T><<<grid_stride_blocks(n), kBlock, 0, s>>>(out, v, n);
}

// explicit instantiations
#define MG_INST(T)                                                                        \
    template void apply<T>(const LevelView<T>&, const T*, const T*, T*, hipStream_t);    \
    template void smooth<T>(const LevelView<T>&, const T*, const T*, T*, T, hipStream_t); \
    template void restrict_residual<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, const T*, T*, hipStream_t);              \
    template void prolong_add<T>(const LevelView<T>&, const TransferView<T>&, const T*,  \
                                 T*, hipStream_t);                                        \
    template void prolong_transpose<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, T*, hipStream_t);                        \
    template void inject_residual_adjoint<T>(const LevelView<T>&, const TransferView<T>&, \
                                             const T*, T*, T*, hipStream_t);              \
    template void smooth_transpose<T>(const LevelView<T>&, const T*, const T*, T*, T*,   \
                                      T*, T, bool, hipStream_t);                          \
    template void adjoint_stencil<T>(const LevelView<T>&, const T*, T*, T, hipStream_t); \
    template void fill<T>(T*, T, long long, hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

template int residual_update<float, float>(const LevelView<double>&, const double*,
                                           const double*, const float*, double*, float*,
                                           double*, hipStream_t);
template int residual_update<double, double>(const LevelView<double>&, const double*,
                                             const double*, const double*, double*,
                                             double*, double*, hipStream_t);
template void cast<double, float>(const double*, float*, long long, hipStream_t);
template void cast<float, double>(const float*, double*, long long, hipStream_t);
template void cast<double, double>(const double*, double*, long long, hipStream_t);

}  // namespace mgk
