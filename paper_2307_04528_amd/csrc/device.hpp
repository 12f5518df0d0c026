// Device-side helpers shared by the kernel files (gfx950).
//
// Mapping. Kernels that walk a vertical column (the Thomas solves, and the
// stencils that need the layers above and below) use one lane per column
// (I, J); a wavefront covers 64 consecutive longitudes of a row, so every
// layer k is one coalesced 256 B (FP32) / 512 B (FP64) access per wavefront.
// Kernels with no sequential dependence in k use one lane per cell.
//
// Latency. A column kernel is a chain of nz dependent steps. The layer loop is
// fully unrolled over a compile-time bucket NZ >= nz and every load is
// unconditional: layer indices are clamped to nz-1, neighbour offsets at the
// poles are clamped to the cell itself (their coefficient in the tables is
// exactly 0), and the top/bottom vertical coefficients are 0; only stores are
// guarded. The Thomas sweeps prefetch explicitly: the loads of the next chunk
// of D layers are issued before the current chunk is solved, with scheduling
// barriers so the compiler neither serialises them nor hoists everything
// (which would spill the per-column registers).
//
// Addressing. Each layer of a per-cell array is a wave-uniform base held in
// scalar registers plus a 32-bit per-lane byte offset (global_load with a
// scalar base). Coefficient tables are read through the constant address
// space; where every wavefront lies inside one latitude row (nI a multiple of
// 64) their index is wave-uniform and they become scalar loads.
//
// L2 locality. The hardware hands block b to XCD b % 8; blocks are remapped
// so that each XCD works on one contiguous range of columns, and the
// latitude neighbours that a stencil re-reads come from the same L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace mgk {
namespace dev {

__device__ __forceinline__ uint32_t logical_block() {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

__device__ __forceinline__ uint32_t global_index() {
    return logical_block() * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ int clampk(int k, int nz) { return k < nz ? k : nz - 1; }

// Element offsets (within one layer) of a column and of its four horizontal
// neighbours; at a pole the missing neighbour is the cell itself. ROWU: every
// wavefront lies inside one latitude row, so the row index is wave-uniform.
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

// Row-aligned segments: a latitude row of nI columns is cut into
// wpr = ceil(nI / 64) segments of up to 64 consecutive columns, and one
// wavefront takes one segment, so the row index is wave-uniform on every
// level (not only where 64 divides nI). Lanes past the end of the row, and
// segments past the last row, are marked invalid; their offsets are clamped
// to a real column so that every load stays in bounds.
struct Seg {
    uint32_t c, w, e, s, n;
    int J;
    bool valid;
};

__device__ __forceinline__ Seg segment(int seg, int nI, int nJ, int wpr) {
    int J = seg / wpr;
    const int i = (seg - J * wpr) * 64 + int(threadIdx.x & 63u);
    Seg r;
    r.valid = J < nJ && i < nI;
    J = J < nJ ? J : nJ - 1;
    const int ic = i < nI ? i : nI - 1;
    const uint32_t col = uint32_t(J) * uint32_t(nI) + uint32_t(ic);
    r.J = J;
    r.c = col;
    r.w = (ic == 0) ? col + uint32_t(nI - 1) : col - 1u;
    r.e = (ic == nI - 1) ? col - uint32_t(nI - 1) : col + 1u;
    r.s = (J > 0) ? col - uint32_t(nI) : col;
    r.n = (J < nJ - 1) ? col + uint32_t(nI) : col;
    return r;
}

inline int segments_per_row(int nI) { return (nI + 63) / 64; }

// Row-tiled segments: the R wavefronts (or wavefront pairs) r = 0..R-1 of
// block b take the same 64-column range of R consecutive rows, so most of
// the latitude neighbours a stencil reads belong to the same block and are
// read at about the same time (from the CU's cache), not by a block that
// runs much earlier or later. Rows past nJ are invalid segments.
__device__ __forceinline__ Seg tiled_segment(int b, int r, int R, int nI, int nJ, int wpr) {
    const int band = b / wpr, s = b - band * wpr;
    return segment((band * R + r) * wpr + s, nI, nJ, wpr);
}
inline int tiled_blocks(int nJ, int wpr, int R) { return ((nJ + R - 1) / R) * wpr; }

// Wavefront w of a block: pair w/2 of the block, bottom (even w) or top.
struct PairOf {
    int pair;
    bool top;
};
__device__ __forceinline__ PairOf pair_of_wave() {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    return {wave >> 1, (wave & 1) != 0};
}

// The same offsets in bytes for element type T (a layer of any per-cell
// array is < 4 GiB).
template <typename T>
struct NbB {
    uint32_t c, w, e, s, n;
    int J;
    __device__ __forceinline__ explicit NbB(const Nb& b)
        : c(b.c * uint32_t(sizeof(T))), w(b.w * uint32_t(sizeof(T))),
          e(b.e * uint32_t(sizeof(T))), s(b.s * uint32_t(sizeof(T))),
          n(b.n * uint32_t(sizeof(T))), J(b.J) {}
    __device__ __forceinline__ explicit NbB(const Seg& b)
        : c(b.c * uint32_t(sizeof(T))), w(b.w * uint32_t(sizeof(T))),
          e(b.e * uint32_t(sizeof(T))), s(b.s * uint32_t(sizeof(T))),
          n(b.n * uint32_t(sizeof(T))), J(b.J) {}
};

// Wave-uniform base of layer kk (layer stride Pb bytes), pinned to scalar
// registers, as a global-address-space pointer.
__device__ __forceinline__ uint64_t uniform64(uint64_t p) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(p));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(p >> 32));
    return (uint64_t(hi) << 32) | lo;
}
typedef const __attribute__((address_space(1))) char* gcptr;
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

// Buffer instructions. A raw buffer resource over `bytes` bytes at p (32-bit
// data format, no stride); an access gives a per-lane byte offset and a
// wave-uniform one, so the per-cell arrays of a level, which share one
// layout, address layer k of any of them with the same scalar offset.
typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, int(bytes),
                                             0x00020000);
}
// Cache policy of the non-temporal hint (bit nt), for loads and stores.
constexpr int kPolicyNT = 2;

// Per-cell fields of at least this many bytes: a kernel's three or four
// such arrays exceed the 256 MB last-level cache at least twice over, so
// what it reads once is not found there again by the next kernel, and those
// loads carry the non-temporal hint. On smaller levels the repeated sweeps
// still find part of their right-hand side there (measured on the
// 512x504x70 level, 72 MB per FP32 field: its sweeps 51 us with plain
// loads, 61 us with the hint; the 1024x768x70 solve 1.9% faster with this
// bound than with 64 MB).
constexpr long long kStreamFieldBytes = 1LL << 27;

// Loads. NT: with the non-temporal hint, for arrays a kernel reads once per
// cell and no neighbouring lane or row reads again (a right-hand side, the
// mass, the pivots), so that they do not take the cache lines of the arrays
// whose latitude neighbours are read again from L2.
template <typename T, bool NT = false>
__device__ __forceinline__ T bld(rsrc_t r, uint32_t voff, uint32_t soff) {
    constexpr int pol = NT ? kPolicyNT : 0;
    if constexpr (std::is_same<T, float>::value)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff),
                                                                              int(soff), pol));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff),
                                                                               int(soff), pol));
}

// Stores, with the non-temporal hint unless NT is false. A kernel never
// reads back what it stores through these; the next kernel reads it. On
// large levels the hint keeps the written field from evicting the lines
// still being read; on levels whose fields stay in the caches between
// kernels it costs the next kernel those hits (measured on the 70-layer
// shells: sweeps of 14M cells or more 2-7% faster with it, sweeps of 3-5M
// cells 10-12% slower).
template <bool NT = true>
__device__ __forceinline__ void bst(float v, rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff),
                                          int(soff), NT ? kPolicyNT : 0);
}
template <bool NT = true>
__device__ __forceinline__ void bst(double v, rsrc_t r, uint32_t voff, uint32_t soff) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, int(voff), int(soff),
                                          NT ? kPolicyNT : 0);
}

// Two adjacent values (a lane's two longitude children) with one load.
template <typename T>
using pair_t = T __attribute__((ext_vector_type(2)));
template <typename T, bool NT = false>
__device__ __forceinline__ pair_t<T> bld2(rsrc_t r, uint32_t voff, uint32_t soff) {
    constexpr int pol = NT ? kPolicyNT : 0;
    if constexpr (std::is_same<T, float>::value)
        return __builtin_bit_cast(pair_t<float>, __builtin_amdgcn_raw_buffer_load_b64(
                                                     r, int(voff), int(soff), pol));
    else
        return __builtin_bit_cast(pair_t<double>, __builtin_amdgcn_raw_buffer_load_b128(
                                                      r, int(voff), int(soff), pol));
}

// Read-only coefficient tables through the constant address space.
template <typename T>
__device__ __forceinline__ T tab(const T* p, int idx) {
    return ((const __attribute__((address_space(4))) T*)p)[idx];
}

// Record i of a step table, through the constant address space (the index
// is wave-uniform: one scalar load).
template <typename T>
__device__ __forceinline__ StepCoef<T> step_rec(const StepCoef<T>* p, size_t i) {
    const __attribute__((address_space(4))) T* q =
        (const __attribute__((address_space(4))) T*)(p + i);
    return {q[0], q[1], q[2], q[3]};
}

// Lane shifts of a wavefront by one lane (DPP wave_shr / wave_shl): lane l
// takes src of lane l-1 (from_below) or l+1 (from_above); the lane with no
// source (0, respectively 63) keeps `edge`.
__device__ __forceinline__ float from_below(float edge, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, src),
                                                                 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_above(float edge, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, src),
                                                                 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_below(double edge, double src) {
    typedef int i2 __attribute__((ext_vector_type(2)));
    const i2 e = __builtin_bit_cast(i2, edge), s = __builtin_bit_cast(i2, src);
    const i2 r = {__builtin_amdgcn_update_dpp(e.x, s.x, 0x138, 0xf, 0xf, false),
                  __builtin_amdgcn_update_dpp(e.y, s.y, 0x138, 0xf, 0xf, false)};
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double from_above(double edge, double src) {
    typedef int i2 __attribute__((ext_vector_type(2)));
    const i2 e = __builtin_bit_cast(i2, edge), s = __builtin_bit_cast(i2, src);
    const i2 r = {__builtin_amdgcn_update_dpp(e.x, s.x, 0x130, 0xf, 0xf, false),
                  __builtin_amdgcn_update_dpp(e.y, s.y, 0x130, 0xf, 0xf, false)};
    return __builtin_bit_cast(double, r);
}

// The value of x in lane l (l wave-uniform).
__device__ __forceinline__ float lane_value(float x, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(u)), l));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(u >> 32)), l));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// One latitude row J of a coefficient table, tab[F * stride + J] for
// F = 0..count-1 (count <= N), spread over the lanes of a wavefront (lane l
// of slot r holds entry 64 r + l) and read back with readlane at a
// wave-uniform index. A column recurrence that reads its couplings this way
// waits on no memory access per layer; through tab() each layer's couplings
// are scalar loads, and every step waits for one.
template <typename T, int N>
struct LaneTable {
    static constexpr int R = (N + 63) / 64;
    T v[R];
    __device__ __forceinline__ LaneTable(const T* tab, int stride, int J, int count) {
        const int lane = int(threadIdx.x & 63u);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int F = r * 64 + lane;
            v[r] = F < count ? tab[size_t(F) * size_t(stride) + size_t(J)] : T(0);
        }
    }
    __device__ __forceinline__ T operator()(int F) const {
        const int l = F & 63, r = F >> 6;
        T x = lane_value(v[0], l);
#pragma unroll
        for (int q = 1; q < R; ++q) {
            const T y = lane_value(v[q], l);
            x = (r == q) ? y : x;
        }
        return x;
    }
};

// Stands in for a LaneTable where the table is read through tab() instead.
template <typename T>
struct NoLaneTable {
    __device__ __forceinline__ NoLaneTable(const T*, int, int, int) {}
};

// Two block sums with one barrier: *out_a = sum of a, *out_b = sum of b.
template <typename T>
__device__ __forceinline__ void block_sum2_to(T a, T b, T* out_a, T* out_b) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    __shared__ T red2[2][1024 / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red2[0][wave] = a;
        red2[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T ta = 0, tb = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) {
            ta += red2[0][w];
            tb += red2[1][w];
        }
        *out_a = ta;
        *out_b = tb;
    }
}

template <typename T>
__device__ __forceinline__ void block_sum_to(T v, T* out) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __shared__ T red[1024 / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) t += red[w];
        *out = t;
    }
}

// Horizontal part of H at one cell in difference form:
// Tlam (2xc - xw - xe) + Ts (xc - xs) + Tn (xc - xn).
template <typename T>
__device__ __forceinline__ T hdiff(T tl, T ts, T tn, T xc, T xw, T xe, T xs, T xn) {
    return tl * ((xc - xw) + (xc - xe)) + ts * (xc - xs) + tn * (xc - xn);
}

}  // namespace dev

inline int grid_stride_blocks(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    return int(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// Dispatch the layer-count bucket NZ >= nz at compile time.
template <typename F>
void with_nz(int nz, F&& fn) {
    if (nz <= 16) fn(std::integral_constant<int, 16>{});
    else if (nz <= 32) fn(std::integral_constant<int, 32>{});
    else if (nz <= 72) fn(std::integral_constant<int, 72>{});
    else fn(std::integral_constant<int, 128>{});
}

// Levels with fewer columns than this run their Thomas sweeps with the
// deeper prefetch (more layers in flight per lane, fewer lanes): below
// ~2^19 columns the GPU holds every column at once, so the per-column
// latency chain, not the bandwidth, sets the time.
constexpr long long kSmallLevelColumns = 1LL << 19;

}  // namespace mgk
