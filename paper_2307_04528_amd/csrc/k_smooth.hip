// Block-Jacobi smoother (paper Eq. 1, Section 2.1) and its transpose.
//
// One sweep, with the vertical couplings in H_z solved exactly per column:
//   x_new = (1 - omega) x + omega H_z^{-1} (f + sum_h T_h x_nb)
// which equals x + omega H_z^{-1}(f - H x) since H = H_z + dH and dH holds
// only the horizontal off-diagonals -T_h. The column solve is the Thomas
// algorithm with precomputed inverse pivots (row-sum form, see setup).
#include "device.hpp"

namespace mgk {

#ifndef MG_SMOOTH_KEEP_P
#define MG_SMOOTH_KEEP_P 0
#endif
#ifndef MG_SMOOTH_WAVES32
#define MG_SMOOTH_WAVES32 2
#endif
#ifndef MG_SMOOTH_WAVES64
#define MG_SMOOTH_WAVES64 1
#endif
#ifndef MG_SMOOTH_KEEP_X
#define MG_SMOOTH_KEEP_X 0
#endif
#ifndef MG_CHUNK32
#define MG_CHUNK32 4
#endif
#ifndef MG_CHUNK64
#define MG_CHUNK64 4
#endif
#ifndef MG_CHUNK_SMALL
#define MG_CHUNK_SMALL 8
#endif

namespace {
using namespace dev;

// Occupancy target (waves per SIMD): caps the registers of a column kernel.
template <typename T>
struct ColumnWaves {
    static constexpr int value = std::is_same<T, float>::value ? MG_SMOOTH_WAVES32
                                                                : MG_SMOOTH_WAVES64;
};
// Layers per prefetch chunk on levels large enough to fill the GPU.
template <typename T>
struct ChunkDepth {
    static constexpr int value = std::is_same<T, float>::value ? MG_CHUNK32 : MG_CHUNK64;
};

// Thomas solve of one column, z = H_z^{-1} s, with chunked prefetch.
//   src(k, kk)            -> s_kk (issues the loads of layer kk)
//   fwd_sink(k, kk, s)    called once s_k is available (e.g. to store it)
//   bload(k, kk, e[NB])   extra per-layer loads needed by the backward sink
//   sink(k, kk, z, e[NB]) consumes z_k, top layer first
// Layers k >= nz (bucket padding) are computed on clamped data and never
// stored.
template <typename T, int NZ, int D, bool KEEP_P, int NB, class Src, class FSink, class BLoad,
          class Sink>
__device__ __forceinline__ void thomas_column(const LevelView<T>& L, int J, uint32_t boff,
                                              Src src, FSink fwd_sink, BLoad bload, Sink sink) {
    const int nJ = L.nJ, nz = L.nz;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    constexpr int NC = (NZ + D - 1) / D;
    T y[NC * D];
    T ip[KEEP_P ? NC * D : 1];
    T bs[2][D], bp[2][D];
    auto load = [&](int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kk = clampk(c * D + d, nz);
            bs[buf][d] = src(c * D + d, kk);
            bp[buf][d] = ldb<T>(layer(L.invp, kk, Pb), boff);
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
            const int k = c * D + d;
            const int kk = clampk(k, nz);
            fwd_sink(k, kk, bs[c & 1][d]);
            yp = (bs[c & 1][d] + tab(L.Tr, kk * nJ + J) * yp) * bp[c & 1][d];
            y[k] = yp;
            if constexpr (KEEP_P) ip[k] = bp[c & 1][d];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    T bq[2][D];
    T be[2][D][NB > 0 ? NB : 1];
    auto load_back = [&](int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kk = clampk(c * D + d, nz);
            if constexpr (!KEEP_P) bq[buf][d] = ldb<T>(layer(L.invp, kk, Pb), boff);
            if constexpr (NB > 0) bload(c * D + d, kk, be[buf][d]);
        }
    };
    T zn = 0;
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
            zn = (k < nz) ? y[k] + tab(L.Tr, (kk + 1) * nJ + J) * p * zn : T(0);
            sink(k, kk, zn, be[c & 1][d]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One forward sweep of one column (see the file comment); xin == nullptr
// (HAS_X false): the sweep from zero, omega H_z^{-1} f.
template <typename T, int NZ, int D, bool HAS_X, bool ROWU>
__device__ __forceinline__ void sweep_column(const LevelView<T>& L, const T* f, const T* xin,
                                             T* xout, T omega, uint32_t col) {
    const NbB<T> b(neighbours<ROWU>(col, L.nI, L.nJ));
    const int nJ = L.nJ, nz = L.nz;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    const T keep = T(1) - omega;
    // KEEP_X: the column's own old value is loaded in the forward pass (its
    // cache lines are those of the east/west neighbours) and kept for the
    // damping term, instead of being fetched again in the backward pass
    constexpr bool KX = HAS_X && MG_SMOOTH_KEEP_X != 0;
    constexpr int NP = ((NZ + D - 1) / D) * D;
    T xkeep[KX ? NP : 1];
    auto src = [&](int k, int kk) -> T {
        T s = ldb<T>(layer(f, kk, Pb), b.c);
        if constexpr (HAS_X) {
            gcptr xk = layer(xin, kk, Pb);
            s += tab(L.Tlam, kk * nJ + b.J) * (ldb<T>(xk, b.w) + ldb<T>(xk, b.e)) +
                 tab(L.Tth, kk * (nJ + 1) + b.J) * ldb<T>(xk, b.s) +
                 tab(L.Tth, kk * (nJ + 1) + b.J + 1) * ldb<T>(xk, b.n);
            if constexpr (KX) xkeep[k] = ldb<T>(xk, b.c);
        }
        return s;
    };
    auto fsink = [&](int, int, T) {};
    auto bload = [&](int, int kk, T (&e)[1]) { e[0] = ldb<T>(layer(xin, kk, Pb), b.c); };
    auto sink = [&](int k, int kk, T z, const T (&e)[1]) {
        T out = omega * z;
        if constexpr (KX) out += keep * xkeep[k];
        else if constexpr (HAS_X) out += keep * e[0];
        if (k < nz) stb<T>(layer_w(xout, kk, Pb), b.c, out);
    };
    thomas_column<T, NZ, D, MG_SMOOTH_KEEP_P != 0, (HAS_X && !KX) ? 1 : 0>(
        L, b.J, b.c, src, fsink, bload, sink);
}

template <typename T, int NZ, int D, bool HAS_X, bool ROWU>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ColumnWaves<T>::value)))
void k_smooth(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ xin,
              T* __restrict__ xout, T omega) {
    const uint32_t col = global_index();
    if (col >= uint32_t(L.plane)) return;
    sweep_column<T, NZ, D, HAS_X, ROWU>(L, f, xin, xout, omega, col);
}

// The coarsest level in one launch: one block does every sweep from zero,
// ping-ponging between xa and xb, with a block barrier between sweeps (the
// global writes of a sweep are visible to the whole block after it). The
// result is in xa if sweeps is odd, else in xb.
template <typename T, int NZ, int D>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(LevelView<T> L, const T* __restrict__ f,
                                                       T* xa, T* xb, T omega, int sweeps) {
    const uint32_t plane = uint32_t(L.plane);
    for (int s = 0; s < sweeps; ++s) {
        T* xout = (s & 1) ? xb : xa;
        const T* xin = (s & 1) ? xa : xb;
        for (uint32_t col = threadIdx.x; col < plane; col += blockDim.x) {
            if (s == 0) sweep_column<T, NZ, D, false, false>(L, f, nullptr, xout, omega, col);
            else sweep_column<T, NZ, D, true, false>(L, f, xin, xout, omega, col);
        }
        __syncthreads();
    }
}

// The coarsest level in one launch with its data in LDS: one lane per column
// (plane <= blockDim); the right-hand side, the inverse pivots and the
// iterate are staged in LDS ([k][col]) once. A sweep reads the old
// neighbours from LDS, with the same chunked prefetch as the other column
// kernels, keeps its new column in the Thomas registers, and after a block
// barrier overwrites the old iterate; a sweep then costs a few microseconds.
// UNIT: block b solves for the b-th unit vector instead of f and writes its
// result to row b of xout (rows of n values): the grid then computes the
// solve's explicit matrix, transposed, one row per block.
template <typename T, int NZ, bool UNIT>
__global__ __launch_bounds__(kBlock) void k_coarse_lds(LevelView<T> L, const T* __restrict__ f,
                                                       T* __restrict__ xout, T omega,
                                                       int sweeps) {
    extern __shared__ unsigned char smem_raw[];
    const int plane = int(L.plane), nz = L.nz, nJ = L.nJ, n = plane * nz;
    if constexpr (UNIT) xout += size_t(blockIdx.x) * size_t(n);
    T* sx = reinterpret_cast<T*>(smem_raw);
    T* sf = sx + n;
    T* sp = sf + n;
    // the coefficient tables too (read from LDS inside the sweep loop, they
    // are not hoisted out of it into registers)
    T* stl = sp + n;                 // [nz][nJ]
    T* sth = stl + nz * nJ;          // [nz][nJ+1]
    T* str = sth + nz * (nJ + 1);    // [nz+1][nJ]
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        sx[t] = T(0);   // the first sweep starts from zero: same code as the rest
        if constexpr (UNIT) sf[t] = (t == int(blockIdx.x)) ? T(1) : T(0);
        else sf[t] = f[t];
        sp[t] = L.invp[t];
    }
    for (int t = threadIdx.x; t < nz * nJ; t += blockDim.x) stl[t] = L.Tlam[t];
    for (int t = threadIdx.x; t < nz * (nJ + 1); t += blockDim.x) sth[t] = L.Tth[t];
    for (int t = threadIdx.x; t < (nz + 1) * nJ; t += blockDim.x) str[t] = L.Tr[t];
    __syncthreads();
    const int col = threadIdx.x;
    const bool active = col < plane;
    const Nb b = neighbours<false>(active ? uint32_t(col) : 0u, L.nI, nJ);
    constexpr int D = MG_CHUNK_SMALL;
    constexpr int NC = (NZ + D - 1) / D;
    const T keep = T(1) - omega;
    T y[NC * D];
    for (int s = 0; s < sweeps; ++s) {
        // opaque copies of the strides: the per-layer LDS addresses are then
        // recomputed each sweep instead of being hoisted out of the sweep
        // loop into hundreds of registers (the empty asm emits nothing)
        int pl = plane, nj = nJ;
        asm volatile("" : "+s"(pl), "+s"(nj));
        if (active) {
            T bs[2][D], bp[2][D];
            auto load = [&](int c, int buf) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int kk = clampk(c * D + d, nz);
                    const T* xk = sx + kk * pl;
                    bs[buf][d] = sf[kk * pl + b.c] +
                                 stl[kk * nj + b.J] * (xk[b.w] + xk[b.e]) +
                                 sth[kk * (nj + 1) + b.J] * xk[b.s] +
                                 sth[kk * (nj + 1) + b.J + 1] * xk[b.n];
                    bp[buf][d] = sp[kk * pl + b.c];
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
                    yp = (bs[c & 1][d] + str[kk * nj + b.J] * yp) * bp[c & 1][d];
                    y[c * D + d] = yp;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            T bx[2][D], bq[2][D], bt[2][D];
            auto load_back = [&](int c, int buf) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int kk = clampk(c * D + d, nz);
                    bx[buf][d] = sx[kk * pl + b.c];
                    bq[buf][d] = sp[kk * pl + b.c];
                    bt[buf][d] = str[(kk + 1) * nj + b.J];
                }
            };
            T zn = 0;
            load_back(NC - 1, (NC - 1) & 1);
#pragma unroll
            for (int c = NC - 1; c >= 0; --c) {
                if (c > 0) load_back(c - 1, (c - 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int d = D - 1; d >= 0; --d) {
                    const int k = c * D + d;
                    zn = (k < nz) ? y[k] + bt[c & 1][d] * bq[c & 1][d] * zn : T(0);
                    y[k] = omega * zn + keep * bx[c & 1][d];   // the new iterate
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // every lane has read the old iterate
        if (active) {
#pragma unroll
            for (int k = 0; k < NZ; ++k)
                if (k < nz) sx[k * plane + b.c] = y[k];
        }
        __syncthreads();   // the new iterate is complete
    }
    if (active) {
#pragma unroll
        for (int k = 0; k < NZ; ++k)
            if (k < nz) xout[size_t(k) * plane + b.c] = y[k];
    }
}

// ---------------------------------------------------------------------------
// Transposed sweep chain kernel:
//   xb' = HAS_Z ? (1-omega) xb + omega sum_h T_h zin_nb : xb   (-> xbout)
//   z = H_z^{-1} xb';  fb = (ACC ? fb : 0) + omega z;  zout = z (if set)
template <typename T, int NZ, int D, bool HAS_Z, bool ACC, bool ROWU>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ColumnWaves<T>::value)))
void k_smooth_T(LevelView<T> L, const T* xb, const T* __restrict__ zin,
                T* xbout,  // may alias xb
                T* __restrict__ zout, T* __restrict__ fb, T omega) {
    const uint32_t col = global_index();
    if (col >= uint32_t(L.plane)) return;
    const NbB<T> b(neighbours<ROWU>(col, L.nI, L.nJ));
    const int nJ = L.nJ, nz = L.nz;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    const T keep = T(1) - omega;
    auto src = [&](int, int kk) -> T {
        T s = ldb<T>(layer(xb, kk, Pb), b.c);
        if constexpr (HAS_Z) {
            gcptr zk = layer(zin, kk, Pb);
            const T h = tab(L.Tlam, kk * nJ + b.J) * (ldb<T>(zk, b.w) + ldb<T>(zk, b.e)) +
                        tab(L.Tth, kk * (nJ + 1) + b.J) * ldb<T>(zk, b.s) +
                        tab(L.Tth, kk * (nJ + 1) + b.J + 1) * ldb<T>(zk, b.n);
            s = keep * s + omega * h;
        }
        return s;
    };
    auto fsink = [&](int k, int kk, T s) {
        if constexpr (HAS_Z) {
            if (k < nz) stb<T>(layer_w(xbout, kk, Pb), b.c, s);
        }
    };
    auto bload = [&](int, int kk, T (&e)[1]) { e[0] = ldb<T>(layer(fb, kk, Pb), b.c); };
    auto sink = [&](int k, int kk, T z, const T (&e)[1]) {
        T fo = omega * z;
        if constexpr (ACC) fo += e[0];
        if (k < nz) {
            if (zout) stb<T>(layer_w(zout, kk, Pb), b.c, z);
            stb<T>(layer_w(fb, kk, Pb), b.c, fo);
        }
    };
    thomas_column<T, NZ, ChunkDepth<T>::value, false, ACC ? 1 : 0>(L, b.J, b.c, src, fsink,
                                                                    bload, sink);
}

// xb = (1-omega) xb + omega sum_h T_h z_nb, one lane per cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint_stencil(LevelView<T> L,
                                                            const T* __restrict__ z,
                                                            T* __restrict__ xb, T omega,
                                                            uint32_t n) {
    const uint32_t t = global_index();
    if (t >= n) return;
    const uint32_t P = uint32_t(L.plane);
    const int k = int(t / P);
    const Nb b = neighbours<false>(t - uint32_t(k) * P, L.nI, L.nJ);
    const int nJ = L.nJ;
    const T* zk = z + size_t(k) * P;
    const T h = L.Tlam[k * nJ + b.J] * (zk[b.w] + zk[b.e]) + L.Tth[k * (nJ + 1) + b.J] * zk[b.s] +
                L.Tth[k * (nJ + 1) + b.J + 1] * zk[b.n];
    xb[t] = (T(1) - omega) * xb[t] + omega * h;
}

}  // namespace

template <typename T>
void smooth(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega, hipStream_t s) {
    const int nb = blocks_for(L.plane);
    const bool small = L.plane < kSmallLevelColumns;
    const bool rowu = L.nI % 64 == 0;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        constexpr int DB = ChunkDepth<T>::value, DS = MG_CHUNK_SMALL;
#define MG_SMOOTH_LAUNCH(D, HX, RU) \
    k_smooth<T, NZ, D, HX, RU><<<nb, kBlock, 0, s>>>(L, f, xin, xout, omega)
        if (small) {
            if (xin) { if (rowu) MG_SMOOTH_LAUNCH(DS, true, true); else MG_SMOOTH_LAUNCH(DS, true, false); }
            else { if (rowu) MG_SMOOTH_LAUNCH(DS, false, true); else MG_SMOOTH_LAUNCH(DS, false, false); }
        } else {
            if (xin) { if (rowu) MG_SMOOTH_LAUNCH(DB, true, true); else MG_SMOOTH_LAUNCH(DB, true, false); }
            else { if (rowu) MG_SMOOTH_LAUNCH(DB, false, true); else MG_SMOOTH_LAUNCH(DB, false, false); }
        }
#undef MG_SMOOTH_LAUNCH
    });
}

// Launch k_coarse_lds<T, NZ, UNIT> on `blocks` blocks; false if the level
// does not fit one block's LDS.
template <typename T, bool UNIT>
bool launch_coarse_lds(const LevelView<T>& L, const T* f, T* x, T omega, int sweeps,
                       size_t max_lds, int blocks, hipStream_t s) {
    const size_t lds = coarse_lds_bytes<T>(L.plane, L.nJ, L.nz);
    if (L.plane > kBlock || lds > max_lds) return false;
    int threads = int(((L.plane + 63) / 64) * 64);
    bool launched = false;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_lds<T, NZ, UNIT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        k_coarse_lds<T, NZ, UNIT><<<blocks, threads, lds, s>>>(L, f, x, omega, sweeps);
        launched = true;
    });
    return launched;
}

template <typename T>
int coarse_solve(const LevelView<T>& L, const T* f, T* xa, T* xb, T omega, int sweeps,
                 size_t max_lds, hipStream_t s) {
    if (launch_coarse_lds<T, false>(L, f, xa, omega, sweeps, max_lds, 1, s)) return 0;
    int threads = int(((L.plane + 63) / 64) * 64);
    if (threads > kBlock) threads = kBlock;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        k_coarse_solve<T, NZ, MG_CHUNK_SMALL><<<1, threads, 0, s>>>(L, f, xa, xb, omega, sweeps);
    });
    return (sweeps & 1) ? 0 : 1;
}

template <typename T>
void smooth_transpose(const LevelView<T>& L, const T* xb, const T* zin, T* xbout, T* zout,
                      T* fb, T omega, bool accumulate, hipStream_t s) {
    const int nb = blocks_for(L.plane);
    const bool rowu = L.nI % 64 == 0;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        constexpr int D = ChunkDepth<T>::value;
#define MG_SMOOTHT_LAUNCH(HZ, AC, RU) \
    k_smooth_T<T, NZ, D, HZ, AC, RU><<<nb, kBlock, 0, s>>>(L, xb, zin, xbout, zout, fb, omega)
        if (zin) {
            if (accumulate) { if (rowu) MG_SMOOTHT_LAUNCH(true, true, true); else MG_SMOOTHT_LAUNCH(true, true, false); }
            else { if (rowu) MG_SMOOTHT_LAUNCH(true, false, true); else MG_SMOOTHT_LAUNCH(true, false, false); }
        } else {
            if (accumulate) { if (rowu) MG_SMOOTHT_LAUNCH(false, true, true); else MG_SMOOTHT_LAUNCH(false, true, false); }
            else { if (rowu) MG_SMOOTHT_LAUNCH(false, false, true); else MG_SMOOTHT_LAUNCH(false, false, false); }
        }
#undef MG_SMOOTHT_LAUNCH
    });
}

template <typename T>
void adjoint_stencil(const LevelView<T>& L, const T* z, T* xb, T omega, hipStream_t s) {
    const long long n = L.plane * L.nz;
    k_adjoint_stencil<T><<<blocks_for(n), kBlock, 0, s>>>(L, z, xb, omega, uint32_t(n));
}

bool coarse_basis(const LevelView<double>& L, double* Ct, double omega, int sweeps,
                  size_t max_lds, hipStream_t s) {
    const long long n = L.plane * L.nz;
    if (n > kDenseCoarseMax || n < 1) return false;
    return launch_coarse_lds<double, true>(L, nullptr, Ct, omega, sweeps, max_lds, int(n), s);
}

#define MG_INST(T)                                                                          \
    template void smooth<T>(const LevelView<T>&, const T*, const T*, T*, T, hipStream_t);   \
    template int coarse_solve<T>(const LevelView<T>&, const T*, T*, T*, T, int, size_t,       \
                                 hipStream_t);                                              \
    template void smooth_transpose<T>(const LevelView<T>&, const T*, const T*, T*, T*, T*, \
                                      T, bool, hipStream_t);                                \
    template void adjoint_stencil<T>(const LevelView<T>&, const T*, T*, T, hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mgk
